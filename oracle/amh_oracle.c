/*
 * CPU oracle for the AMHMVS checkerboard PatchMatch pass (arXiv 1805.07920).
 *
 * TEST INFRASTRUCTURE ONLY: a plain double-precision restatement of the
 * method that the GPU library is checked against.  Nothing in the library
 * calls, links or loads it.  Every function cites the part of the paper it
 * follows; where the paper is silent or garbled the reading used is named
 * (R0..R14) and listed with its justification in the design notes.
 *
 * Readings used here:
 *   R0  images are grayscale on [0,255]; pixel centres at integer (x,y); depth
 *       is camera z; X_cam = R X_world + t; red = (x+y) even, updated first.
 *   R1  initial cost of a random plane = mean of the k lowest per-view costs
 *       (the best-K heuristic the paper recalls in its related work).
 *   R2  region geometry of the asymmetric propagation (the figure that fixes it
 *       is missing): near regions are V-shaped wedges of 7 pixels, far regions
 *       are axial strips of 11 pixels at odd distances 3..23.
 *   R3  a hypothesis costs 2 if its depth at the pixel is outside
 *       [d_min, d_max] (by more than a relative 1e-5), if the window centre
 *       does not project inside the source image, or if any window sample's
 *       ray meets the plane behind the reference camera or lands behind the
 *       source camera.
 *   R4  the window is 11x11 sampled at every other row and column: offsets
 *       {-5,-3,-1,1,3,5}^2, 36 samples.
 *   R5  bilateral weight exp(-|dI|/(2 sI^2) - |dx|/(2 sx^2)) with the colour
 *       difference and the spatial distance unsquared, as the paper prints it;
 *       weights come from the reference patch and apply to both patches.
 *       bilateral_sq = 1 takes the usual squared form exp(-dI^2/(2 sI^2) -
 *       |dx|^2/(2 sx^2)) instead.
 *   R6  a patch with weighted variance below 1e-5 gives cost 2.
 *   R7  the pixel's current plane is scored as a ninth row, excluded from the
 *       view inference, included in the final argmin (ties keep it).
 *   R8  t is the 0-based iteration, the same for the red and the black pass.
 *   R9  the good-view test uses strict inequalities.
 *   R10 v_t is the argmax of the unmodified importance over S_t (lowest index
 *       on ties), -1 if S_t is empty.
 *   R11 the doubled importance goes to v_{t-1} when it is in S_t; the k views
 *       with the largest modified importance keep it as weight; views of
 *       S_{t-1} that left S_t weigh 0.2; every other view weighs 0.
 *   R12 if every weight is 0 the cost is the plain mean over all views.
 *   R13 refinement: perturbed depth/normal candidates in the first 3
 *       iterations, plus random ones afterwards; strictly lower cost wins.
 *   R15 symmetric checkerboard propagation of the ablation (the figure that
 *       fixes Gipuma's patterns is missing): the fast version, 8 fixed
 *       neighbours at distances 1 and 5 up/down/left/right, one per row of the
 *       8-row cost matrix, so the joint view selection sees the same shape.
 *   R16 heuristic view selection of the ablation: each hypothesis (and each
 *       refinement candidate) costs the mean of its own k lowest per-view
 *       costs; no view-selection memory is kept (S = 0, v = -1).
 */
#include "amh_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x64 with 10 rounds, as published by  */
/* Salmon, Moraes, Dror and Shaw (SC'11).  Keyed by the seed; the counter     */
/* carries (pixel index, iteration, purpose, 0).                              */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform in [0,1) from the top 24 bits of a 64-bit word (exact in float and double) */
double orc_u24(uint64_t w) { return (double)(w >> 40) * (1.0 / 16777216.0); }

static void draw4(const orc_params *p, uint64_t pix, uint64_t t, uint64_t purpose, double u[4])
{
    uint64_t ctr[4] = {pix, t, purpose, 0}, key[2] = {p->seed, 0}, w[4];
    orc_philox4x64_10(ctr, key, w);
    for (int i = 0; i < 4; ++i) u[i] = orc_u24(w[i]);
}

/* ------------------------------------------------------------------------ */
/* Asymmetric checkerboard propagation regions (Sec. 3.1, Fig. 2(d), R2).     */
/* 4 near regions of 7 candidates and 4 far regions of 11 candidates, in the  */
/* order up, down, left, right (near first).                                  */
/* ------------------------------------------------------------------------ */
int orc_acp_offsets(int *dx, int *dy, int *region)
{
    /* the "up" member of each family, as (dx, dy) with y pointing down */
    int near_up[7][2] = {{0, -1}, {-1, -2}, {1, -2}, {-2, -3}, {2, -3}, {-3, -4}, {3, -4}};
    int far_up[11][2];
    for (int m = 0; m < 11; ++m) { far_up[m][0] = 0; far_up[m][1] = -(3 + 2 * m); }
    int n = 0;
    for (int fam = 0; fam < 2; ++fam) {
        int cnt = fam == 0 ? 7 : 11;
        for (int dir = 0; dir < 4; ++dir) {
            for (int e = 0; e < cnt; ++e) {
                int ux = fam == 0 ? near_up[e][0] : far_up[e][0];
                int uy = fam == 0 ? near_up[e][1] : far_up[e][1];
                int ox, oy;
                if (dir == 0) { ox = ux; oy = uy; }        /* up */
                else if (dir == 1) { ox = ux; oy = -uy; }  /* down */
                else if (dir == 2) { ox = uy; oy = ux; }   /* left */
                else { ox = -uy; oy = ux; }                /* right */
                dx[n] = ox; dy[n] = oy; region[n] = fam * 4 + dir;
                ++n;
            }
        }
    }
    return n;
}

/* Symmetric checkerboard propagation of the ablation (Sec. 3.1, Fig. 2(c),  */
/* Sec. 4; R15): region r holds the single neighbour at distance 1 (r < 4) or */
/* 5 (r >= 4) in direction up, down, left, right.                             */
int orc_scp_offsets(int *dx, int *dy, int *region)
{
    for (int r = 0; r < 8; ++r) {
        int u = r < 4 ? 1 : 5, dir = r & 3;
        dx[r] = dir == 2 ? -u : (dir == 3 ? u : 0);
        dy[r] = dir == 0 ? -u : (dir == 1 ? u : 0);
        region[r] = r;
    }
    return 8;
}

/* Symmetric checkerboard propagation, standard version (Sec. 3.1, Fig. 2(b),  */
/* Sec. 4; R15): every other-colour pixel within L1 distance 3 and the four    */
/* axial pixels at distance 5, each its own region (20 rows).                  */
int orc_sscp_offsets(int *dx, int *dy, int *region)
{
    int n = 0;
    for (int oy = -5; oy <= 5; ++oy)
        for (int ox = -5; ox <= 5; ++ox) {
            int l1 = abs(ox) + abs(oy);
            if (!(l1 & 1)) continue; /* the other colour */
            if (l1 <= 3 || (l1 == 5 && (ox == 0 || oy == 0))) {
                dx[n] = ox; dy[n] = oy; region[n] = n;
                ++n;
            }
        }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Geometry (R0).                                                             */
/* ------------------------------------------------------------------------ */
static void inv3(const double a[9], double o[9])
{
    double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    o[0] = c00 / det; o[1] = (a[2] * a[7] - a[1] * a[8]) / det; o[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    o[3] = c01 / det; o[4] = (a[0] * a[8] - a[2] * a[6]) / det; o[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    o[6] = c02 / det; o[7] = (a[1] * a[6] - a[0] * a[7]) / det; o[8] = (a[0] * a[4] - a[1] * a[3]) / det;
}

static void mv3(const double m[9], const double v[3], double o[3])
{
    o[0] = m[0] * v[0] + m[1] * v[1] + m[2] * v[2];
    o[1] = m[3] * v[0] + m[4] * v[1] + m[5] * v[2];
    o[2] = m[6] * v[0] + m[7] * v[1] + m[8] * v[2];
}

static void ray_of(const orc_views *V, double sx, double sy, double r[3])
{
    double Kinv[9], q[3] = {sx, sy, 1.0};
    inv3(V->Kref, Kinv);
    mv3(Kinv, q, r);
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Point where the ray of reference pixel (sx, sy) meets the plane, seen by
 * source j: homogeneous pixel coordinates (u*z, v*z, z).  Scene-space planes,
 * no rectification (Sec. 2, 3.3): ray-plane intersection then projection. */
void orc_project(const orc_views *V, double sx, double sy, const double plane[4], int j, double out[3])
{
    double r[3];
    ray_of(V, sx, sy, r);
    double lam = -plane[3] / dot3(plane, r);
    double Xr[3] = {lam * r[0], lam * r[1], lam * r[2]};
    double d[3] = {Xr[0] - V->tref[0], Xr[1] - V->tref[1], Xr[2] - V->tref[2]};
    double Xw[3];  /* R_ref^T (X_ref - t_ref) */
    Xw[0] = V->Rref[0] * d[0] + V->Rref[3] * d[1] + V->Rref[6] * d[2];
    Xw[1] = V->Rref[1] * d[0] + V->Rref[4] * d[1] + V->Rref[7] * d[2];
    Xw[2] = V->Rref[2] * d[0] + V->Rref[5] * d[1] + V->Rref[8] * d[2];
    double Xj[3];
    mv3(V->Rsrc[j], Xw, Xj);
    Xj[0] += V->tsrc[j][0]; Xj[1] += V->tsrc[j][1]; Xj[2] += V->tsrc[j][2];
    mv3(V->Ksrc[j], Xj, out);
}

static double depth_at(const orc_views *V, int x, int y, const double plane[4])
{
    double r[3];
    ray_of(V, x, y, r);
    return -plane[3] / dot3(plane, r);
}

static double ref_at(const orc_views *V, int x, int y)
{
    if (x < 0) x = 0;
    if (x > V->W - 1) x = V->W - 1;
    if (y < 0) y = 0;
    if (y > V->H - 1) y = V->H - 1;
    return V->ref[(long)y * V->W + x];
}

/* bilinear interpolation with clamp-to-edge texel indices */
static double bilinear(const float *img, int W, int H, double px, double py)
{
    if (!(px > -1e9)) px = -1e9;
    if (!(px < 1e9)) px = 1e9;
    if (!(py > -1e9)) py = -1e9;
    if (!(py < 1e9)) py = 1e9;
    double fx0 = floor(px), fy0 = floor(py);
    double fx = px - fx0, fy = py - fy0;
    long x0 = (long)fx0, y0 = (long)fy0, x1 = x0 + 1, y1 = y0 + 1;
    x0 = x0 < 0 ? 0 : (x0 > W - 1 ? W - 1 : x0);
    x1 = x1 < 0 ? 0 : (x1 > W - 1 ? W - 1 : x1);
    y0 = y0 < 0 ? 0 : (y0 > H - 1 ? H - 1 : y0);
    y1 = y1 < 0 ? 0 : (y1 > H - 1 ? H - 1 : y1);
    double i00 = img[y0 * W + x0], i10 = img[y0 * W + x1], i01 = img[y1 * W + x0], i11 = img[y1 * W + x1];
    return (1.0 - fy) * ((1.0 - fx) * i00 + fx * i10) + fy * ((1.0 - fx) * i01 + fx * i11);
}

/* Conditioning probe (not the method): the bilinear interpolant's gradient   */
/* at (px, py), same texels and clamping as bilinear().                        */
static void bilinear_grad(const float *img, int W, int H, double px, double py, double *gx, double *gy)
{
    double fx0 = floor(px), fy0 = floor(py);
    double fx = px - fx0, fy = py - fy0;
    long x0 = (long)fx0, y0 = (long)fy0, x1 = x0 + 1, y1 = y0 + 1;
    x0 = x0 < 0 ? 0 : (x0 > W - 1 ? W - 1 : x0);
    x1 = x1 < 0 ? 0 : (x1 > W - 1 ? W - 1 : x1);
    y0 = y0 < 0 ? 0 : (y0 > H - 1 ? H - 1 : y0);
    y1 = y1 < 0 ? 0 : (y1 > H - 1 ? H - 1 : y1);
    double i00 = img[y0 * W + x0], i10 = img[y0 * W + x1], i01 = img[y1 * W + x0], i11 = img[y1 * W + x1];
    *gx = (1.0 - fy) * (i10 - i00) + fy * (i11 - i01);
    *gy = (1.0 - fx) * (i01 - i00) + fx * (i11 - i10);
}

/* half a float32 ulp of |v| (0 for v = 0) */
static double half_ulp_f32(double v)
{
    return v == 0.0 ? 0.0 : ldexp(1.0, ilogb(v) - 24);
}

/* Conditioning probe (not the method): a deterministic offset uniform in     */
/* [-1/2, 1/2) for a (pixel, view, plane), from a 64-bit mix of their bits.   */
static double probe_noise(int x, int y, int j, const double plane[4])
{
    uint64_t h = (uint64_t)(uint32_t)x * 0x9E3779B97F4A7C15ULL ^ (uint64_t)(uint32_t)y * 0xC2B2AE3D27D4EB4FULL ^
                 (uint64_t)(uint32_t)j * 0x165667B19E3779F9ULL;
    for (int i = 0; i < 4; ++i) {
        uint64_t bits;
        memcpy(&bits, &plane[i], sizeof bits);
        h = (h ^ bits) * 0xD6E8FEB86659FD93ULL;
        h ^= h >> 32;
    }
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ULL;
    h ^= h >> 32;
    return (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

/* ------------------------------------------------------------------------ */
/* Matching cost m(p, h(p)): bilaterally weighted NCC over the window,        */
/* every other row and column (Sec. 3.3, Eq. 8; R3-R6).                       */
/* ------------------------------------------------------------------------ */
double orc_matching_cost(const orc_views *V, const orc_params *p, int x, int y, const double plane[4], int j)
{
    double depth = depth_at(V, x, y, plane);
    /* the range test tolerates a relative 1e-5, so that planes built at a clamped end of the
       range (refinement) are not rejected by the last bit of their reconstruction (R3) */
    if (!(depth > 0.0) || depth < p->d_min * (1.0 - 1e-5) || depth > p->d_max * (1.0 + 1e-5)) return 2.0;
    double c[3];
    orc_project(V, x, y, plane, j, c);
    if (!(c[2] > 0.0)) return 2.0;
    double cu = c[0] / c[2], cv = c[1] / c[2];
    if (!(cu >= 0.0 && cu <= V->srcW[j] - 1 && cv >= 0.0 && cv <= V->srcH[j] - 1)) return 2.0;

    double a[36], b[36], w[36], eb3[36];
    double ac = ref_at(V, x, y);
    int n = 0;
    for (int dy = -5; dy <= 5; dy += 2) {
        for (int dx = -5; dx <= 5; dx += 2) {
            a[n] = ref_at(V, x + dx, y + dy);
            double dcol = fabs(a[n] - ac);
            double dsp = sqrt((double)(dx * dx + dy * dy));
            if (p->bilateral_sq) { dcol *= dcol; dsp *= dsp; } /* the squared form (R5 alternative) */
            w[n] = dcol / (2.0 * p->sigma_color * p->sigma_color) + dsp / (2.0 * p->sigma_spatial * p->sigma_spatial);
            /* every sample's ray must meet the plane in front of the reference camera and the
               point must lie in front of the source camera (R3) */
            double rs[3];
            ray_of(V, x + dx, y + dy, rs);
            if (!(-plane[3] / dot3(plane, rs) > 0.0)) return 2.0;
            double h[3];
            orc_project(V, x + dx, y + dy, plane, j, h);
            if (!(h[2] > 0.0)) return 2.0;
            double px = h[0] / h[2], py = h[1] / h[2];
            if (p->sample_f32 == 1 || p->sample_f32 == 2) { /* conditioning probe only: positions relative to the centre's texel */
                px = floor(cu) + (double)(float)(px - floor(cu));
                py = floor(cv) + (double)(float)(py - floor(cv));
            }
            b[n] = bilinear(V->src[j], V->srcW[j], V->srcH[j], px, py);
            if (p->sample_f32 == 3) { /* conditioning probe only: first-order float32 error bound of b */
                double gx, gy;
                bilinear_grad(V->src[j], V->srcW[j], V->srcH[j], px, py, &gx, &gy);
                eb3[n] = fabs(gx) * half_ulp_f32(px - floor(cu)) + fabs(gy) * half_ulp_f32(py - floor(cv)) +
                         half_ulp_f32(b[n]);
            }
            if (p->sample_f32 == 1 || p->sample_f32 == 2) b[n] = (double)(float)b[n]; /* conditioning probe only */
            ++n;
        }
    }
    /* weights exp(-exponent), scaled by exp(min exponent): a common factor, which cancels in the NCC,
       keeps the largest weight at 1 so that the sum cannot underflow */
    double emin = w[0];
    for (int i = 1; i < 36; ++i) emin = fmin(emin, w[i]);
    for (int i = 0; i < 36; ++i) w[i] = exp(emin - w[i]);
    /* weighted means, then weighted covariances (plain two-pass definition) */
    double sw = 0, sa = 0, sb = 0;
    for (int i = 0; i < 36; ++i) { sw += w[i]; sa += w[i] * a[i]; sb += w[i] * b[i]; }
    double ea = sa / sw, eb = sb / sw;
    double caa = 0, cbb = 0, cab = 0;
    for (int i = 0; i < 36; ++i) {
        caa += w[i] * (a[i] - ea) * (a[i] - ea);
        cbb += w[i] * (b[i] - eb) * (b[i] - eb);
        cab += w[i] * (a[i] - ea) * (b[i] - eb);
    }
    caa /= sw; cbb /= sw; cab /= sw;
    if (p->sample_f32 == 3 && caa > 0.0 && cbb > 0.0) {
        /* conditioning probe only: every sample value moved by the first-order bound of rounding its
           position (relative to the centre's texel) and its value to float32, each in the direction that
           moves the cost towards 1 (the worst case of that rounding, to first order) */
        const double s0 = sqrt(caa * cbb), m0 = 1.0 - cab / s0;
        for (int i = 0; i < 36; ++i) {
            /* dm/db_i: d cab = w (a - ea) / sw, d cbb = 2 w (b - eb) / sw (the mean shifts cancel) */
            const double g = -(w[i] * (a[i] - ea) / sw) / s0 + cab * (w[i] * (b[i] - eb) / sw) / (s0 * cbb);
            b[i] += (m0 >= 1.0) == (g > 0.0) ? -eb3[i] : eb3[i];
        }
        sb = 0;
        for (int i = 0; i < 36; ++i) sb += w[i] * b[i];
        eb = sb / sw;
        cbb = 0; cab = 0;
        for (int i = 0; i < 36; ++i) {
            cbb += w[i] * (b[i] - eb) * (b[i] - eb);
            cab += w[i] * (a[i] - ea) * (b[i] - eb);
        }
        cbb /= sw; cab /= sw;
    }
    if (p->sample_f32 == 2) {
        /* conditioning probe only: the same two-pass definition with weights, sums and moments in
           float32 (this file is compiled without contraction, so every operation rounds once) */
        float swf = 0.f, saf = 0.f, sbf = 0.f;
        for (int i = 0; i < 36; ++i) {
            const float wi = (float)w[i];
            swf += wi;
            saf += wi * (float)a[i];
            sbf += wi * (float)b[i];
        }
        const float eaf = saf / swf, ebf = sbf / swf;
        float caaf = 0.f, cbbf = 0.f, cabf = 0.f;
        for (int i = 0; i < 36; ++i) {
            const float wi = (float)w[i], da = (float)a[i] - eaf, db = (float)b[i] - ebf;
            caaf += wi * da * da;
            cbbf += wi * db * db;
            cabf += wi * da * db;
        }
        caa = caaf / swf;
        cbb = cbbf / swf;
        cab = cabf / swf;
    }
    if (caa < 1e-5 || cbb < 1e-5) return 2.0;
    double m = 1.0 - cab / sqrt(caa * cbb);
    if (p->cost_noise > 0.0) m += probe_noise(x, y, j, plane) * p->cost_noise; /* conditioning probe only */
    if (m < 0.0) m = 0.0;
    if (m > 2.0) m = 2.0;
    return m;
}

/* ------------------------------------------------------------------------ */
/* Multi-hypothesis joint view selection (Sec. 3.2, Eq. 2-6; R8-R12).         */
/* M is row-major [8][N] over the propagated hypotheses.                      */
/* ------------------------------------------------------------------------ */
double orc_tau(const orc_params *p, int t) { return p->tau_mc_init * exp(-(double)t * t / p->alpha); }

static double confidence(const orc_params *p, double m) { return exp(-m * m / (2.0 * p->beta * p->beta)); }

/* The good-view counts n1, n2 are stated for the 8 rows of the method's matrix; with R rows they are
   compared as the same fractions of the rows, n R / 8 (R15). */
void orc_view_selection_rows(const orc_params *p, int t, const double *M, const int *row_valid, int R, int N,
                             uint32_t S_prev, int v_prev, uint32_t *S_out, int *v_out, double *w_out)
{
    double tau = orc_tau(p, t);
    const double n1 = p->n1 * (double)R / 8.0, n2 = p->n2 * (double)R / 8.0;
    int nv = 0;
    for (int i = 0; i < R; ++i) nv += row_valid[i] ? 1 : 0;
    uint32_t S = 0;
    double psi[ORC_MAX_SRC];
    for (int j = 0; j < N; ++j) {
        int lt = 0, gt = 0;
        double sc = 0;
        for (int i = 0; i < R; ++i) {
            if (!row_valid[i]) continue;
            double m = M[i * N + j];
            if (m < tau) ++lt;
            if (m > p->tau_up) ++gt;
            sc += confidence(p, m);
        }
        psi[j] = 0.0;
        if (nv > 0 && lt > n1 && gt < n2) {
            S |= 1u << j;
            psi[j] = sc / nv;
        }
    }
    int v = -1;
    for (int j = 0; j < N; ++j)
        if ((S >> j) & 1u)
            if (v < 0 || psi[j] > psi[v]) v = j;
    double mod[ORC_MAX_SRC];
    for (int j = 0; j < N; ++j) mod[j] = ((S >> j) & 1u) ? (j == v_prev ? 2.0 : 1.0) * psi[j] : 0.0;
    /* keep at most k views of S_t, largest modified importance first, ties to the lower index */
    int keep[ORC_MAX_SRC] = {0};
    for (int r = 0; r < p->k; ++r) {
        int best = -1;
        for (int j = 0; j < N; ++j) {
            if (!((S >> j) & 1u) || keep[j]) continue;
            if (best < 0 || mod[j] > mod[best]) best = j;
        }
        if (best < 0) break;
        keep[best] = 1;
    }
    double sum = 0.0;
    for (int j = 0; j < N; ++j) {
        double wj = 0.0;
        if (keep[j]) wj = mod[j];
        else if (!((S >> j) & 1u) && ((S_prev >> j) & 1u)) wj = 0.2;
        w_out[j] = wj;
        sum += wj;
    }
    if (sum == 0.0)
        for (int j = 0; j < N; ++j) w_out[j] = 1.0;
    *S_out = S;
    *v_out = v;
}

void orc_view_selection(const orc_params *p, int t, const double *M, const int *row_valid, int N,
                        uint32_t S_prev, int v_prev, uint32_t *S_out, int *v_out, double *w_out)
{
    orc_view_selection_rows(p, t, M, row_valid, 8, N, S_prev, v_prev, S_out, v_out, w_out);
}

/* Robustness of the view-selection decisions to perturbations of size delta
 * in M, as bits: ORC_ROBUST_S (the good-view tests), ORC_ROBUST_V (the argmax
 * v_t), ORC_ROBUST_TOPK (the top-k cut).  A good-view test that can flip
 * changes the weights, so it clears every bit. */
static int view_selection_robust(const orc_params *p, int t, const double *M, const int *row_valid, int R, int N,
                                 uint32_t S, int v_prev, double delta)
{
    double tau = orc_tau(p, t);
    double dpsi = 2.1 * delta;  /* |dC/dm| <= 1/(beta sqrt(e)) ~ 2.02 */
    const double n1 = p->n1 * (double)R / 8.0, n2 = p->n2 * (double)R / 8.0;
    int nv = 0;
    for (int i = 0; i < R; ++i) nv += row_valid[i] ? 1 : 0;
    double psi[ORC_MAX_SRC];
    for (int j = 0; j < N; ++j) {
        int lt_lo = 0, lt_hi = 0, gt_lo = 0, gt_hi = 0;
        double sc = 0;
        for (int i = 0; i < R; ++i) {
            if (!row_valid[i]) continue;
            double m = M[i * N + j];
            lt_lo += m < tau - delta;
            lt_hi += m < tau + delta;
            gt_lo += m > p->tau_up + delta;
            gt_hi += m > p->tau_up - delta;
            sc += confidence(p, m);
        }
        int can_true = lt_hi > n1 && gt_lo < n2;
        int can_false = !(lt_lo > n1 && gt_hi < n2);
        if (nv > 0 && can_true && can_false) return 0;
        psi[j] = nv > 0 ? sc / nv : 0.0;
    }
    int bits = ORC_ROBUST_S | ORC_ROBUST_V | ORC_ROBUST_TOPK;
    double mods[ORC_MAX_SRC];
    double top1 = -1.0, top2 = -1.0;
    int n = 0;
    for (int j = 0; j < N; ++j) {
        if (!((S >> j) & 1u)) continue;
        mods[n++] = (j == v_prev ? 2.0 : 1.0) * psi[j];
        if (psi[j] > top1) { top2 = top1; top1 = psi[j]; }
        else if (psi[j] > top2) top2 = psi[j];
    }
    if (n >= 2 && top1 - top2 < 2 * dpsi) bits &= ~ORC_ROBUST_V;
    if (n > p->k) {
        /* gap between the k-th and (k+1)-th modified importance */
        double s[ORC_MAX_SRC];
        memcpy(s, mods, sizeof(double) * (size_t)n);
        for (int a = 0; a < n; ++a)
            for (int b = a + 1; b < n; ++b)
                if (s[b] > s[a]) { double tmp = s[a]; s[a] = s[b]; s[b] = tmp; }
        if (s[p->k - 1] - s[p->k] < 4 * dpsi) bits &= ~ORC_ROBUST_TOPK;
    }
    return bits;
}

/* ------------------------------------------------------------------------ */
/* Random hypotheses (PatchMatch random initialisation, Sec. 2; R13).         */
/* depth uniform in [d_min, d_max], normal uniform on the sphere, turned to  */
/* face the reference camera.                                                 */
/* ------------------------------------------------------------------------ */
static void normal_from_uniforms(double u1, double u2, double n[3])
{
    double z = 1.0 - 2.0 * u1;
    double s = sqrt(fmax(0.0, 1.0 - z * z));
    double phi = 2.0 * 3.14159265358979323846 * u2;
    n[0] = s * cos(phi); n[1] = s * sin(phi); n[2] = z;
}

static void plane_from(const double r[3], double depth, const double nin[3], double plane[4])
{
    double n[3] = {nin[0], nin[1], nin[2]};
    if (dot3(n, r) > 0.0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
    plane[0] = n[0]; plane[1] = n[1]; plane[2] = n[2];
    plane[3] = -depth * dot3(n, r);
}

void orc_random_plane(const orc_views *V, const orc_params *p, int x, int y, uint64_t t, uint64_t purpose,
                      double plane[4])
{
    double u[4], r[3], n[3];
    draw4(p, (uint64_t)y * V->W + x, t, purpose, u);
    ray_of(V, x, y, r);
    double depth = p->d_min + u[0] * (p->d_max - p->d_min);
    normal_from_uniforms(u[1], u[2], n);
    plane_from(r, depth, n, plane);
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* random plane per pixel; initial cost by reading R1; empty selection memory */
void orc_init(const orc_views *V, const orc_params *p, orc_state *s)
{
    long P = (long)V->W * V->H;
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < P; ++i) {
        int x = (int)(i % V->W), y = (int)(i / V->W);
        double plane[4], c[ORC_MAX_SRC];
        orc_random_plane(V, p, x, y, 0, 0, plane);
        for (int j = 0; j < V->n_src; ++j) c[j] = orc_matching_cost(V, p, x, y, plane, j);
        qsort(c, V->n_src, sizeof(double), cmp_double);
        int kk = p->k < V->n_src ? p->k : V->n_src;
        double sum = 0;
        for (int j = 0; j < kk; ++j) sum += c[j];
        memcpy(&s->plane[i * 4], plane, sizeof(plane));
        s->cost[i] = sum / kk;
        s->S[i] = 0;
        s->v[i] = -1;
    }
}

/* ------------------------------------------------------------------------ */
/* One half-pass of the checkerboard (Sec. 3.1-3.3): every pixel of the given */
/* colour picks 8 hypotheses from its asymmetric regions, scores them (plus   */
/* its own) on every source, infers view weights jointly, keeps the best and  */
/* refines it.  Updates in place; reads only the other colour and the pixel   */
/* itself, so the order of the pixels does not matter.                        */
/* ------------------------------------------------------------------------ */
static double mean_k_lowest(const double *c, int n, int k)
{
    double tmp[ORC_MAX_SRC];
    memcpy(tmp, c, sizeof(double) * (size_t)n);
    qsort(tmp, (size_t)n, sizeof(double), cmp_double);
    int kk = k < n ? k : n;
    double sum = 0;
    for (int j = 0; j < kk; ++j) sum += tmp[j];
    return sum / kk;
}

static void update_pixel(const orc_views *V, const orc_params *p, orc_state *s, int t, long idx,
                         const int *odx, const int *ody, const int *oreg, int n_off, double delta, orc_diag *dg)
{
    const int N = V->n_src;
    const int R = p->prop_mode == 2 ? 20 : 8; /* propagated rows; row R is the pixel's own plane */
    int x = (int)(idx % V->W), y = (int)(idx / V->W);
    double planes[ORC_MAX_ROWS][4];
    int valid[ORC_MAX_ROWS];
    int cidx[ORC_MAX_ROWS - 1];
    /* checkerboard propagation: per region, the neighbour with the lowest current cost
       (one neighbour per region in the symmetric patterns) */
    for (int r = 0; r < R; ++r) {
        int best = -1;
        double bc = 0;
        for (int e = 0; e < n_off; ++e) {
            if (oreg[e] != r) continue;
            int nx = x + odx[e], ny = y + ody[e];
            if (nx < 0 || nx >= V->W || ny < 0 || ny >= V->H) continue;
            double c = s->cost[(long)ny * V->W + nx];
            if (best < 0 || c < bc) { best = e; bc = c; }
        }
        cidx[r] = best;
        valid[r] = best >= 0;
        if (valid[r]) memcpy(planes[r], &s->plane[((long)(y + ody[best]) * V->W + (x + odx[best])) * 4], 4 * sizeof(double));
    }
    memcpy(planes[R], &s->plane[idx * 4], 4 * sizeof(double));
    valid[R] = p->include_self ? 1 : 0;

    /* cost matrix (Eq. 1) plus the self row */
    double M[ORC_MAX_ROWS][ORC_MAX_SRC];
    for (int r = 0; r <= R; ++r)
        for (int j = 0; j < N; ++j)
            M[r][j] = valid[r] ? orc_matching_cost(V, p, x, y, planes[r], j) : 2.0;

    double Mflat[(ORC_MAX_ROWS - 1) * ORC_MAX_SRC];
    for (int r = 0; r < R; ++r)
        for (int j = 0; j < N; ++j) Mflat[r * N + j] = M[r][j];
    uint32_t S;
    int v;
    double w[ORC_MAX_SRC];
    orc_view_selection_rows(p, t, Mflat, valid, R, N, s->S[idx], s->v[idx], &S, &v, w);
    if (p->view_mode != 0) {
        S = 0;
        v = -1;
        for (int j = 0; j < N; ++j) w[j] = 1.0;
    }
    const int heuristic = p->view_mode == 2;

    /* unified cost of every hypothesis (Eq. 7; R16 in the heuristic mode) and the minimum;
       ties keep self, then region order */
    double sw = 0;
    for (int j = 0; j < N; ++j) sw += w[j];
    double mf[ORC_MAX_ROWS];
    for (int r = 0; r <= R; ++r) {
        mf[r] = INFINITY;
        if (!valid[r]) continue;
        if (heuristic) { mf[r] = mean_k_lowest(M[r], N, p->k); continue; }
        double acc = 0;
        for (int j = 0; j < N; ++j) acc += w[j] * M[r][j];
        mf[r] = acc / sw;
    }
    int best = -1;
    for (int q = 0; q <= R; ++q) {
        int r = q == 0 ? R : q - 1; /* self first, then the regions in order */
        if (!valid[r]) continue;
        if (best < 0 || mf[r] < mf[best]) best = r;
    }
    double cur[4];
    memcpy(cur, planes[best], sizeof(cur));
    double cur_cost = mf[best];
    int chosen = best;
    int robust = (p->view_mode != 0 ? ORC_ROBUST_S | ORC_ROBUST_V | ORC_ROBUST_TOPK
                                     : view_selection_robust(p, t, Mflat, valid, R, N, S, s->v[idx], delta)) |
                 ORC_ROBUST_ARGMIN | ORC_ROBUST_REFINE;
    if (!(robust & ORC_ROBUST_S)) robust = 0;
    for (int r = 0; r <= R; ++r)
        if (valid[r] && r != best && fabs(mf[r] - mf[best]) < 4 * delta &&
            memcmp(planes[r], planes[best], sizeof(planes[r])) != 0)
            robust &= ~ORC_ROBUST_ARGMIN; /* identical planes tie exactly on any implementation */

    /* refinement (R13) */
    int n_cand = 0;
    double cand[6][4], cand_cost[6];
    if (p->refine) {
        double rr[3];
        ray_of(V, x, y, rr);
        double dcur = -cur[3] / dot3(cur, rr);
        double ncur[3] = {cur[0], cur[1], cur[2]};
        double rho = ldexp(1.0, -(t + 2));
        double ua[4];
        draw4(p, (uint64_t)idx, (uint64_t)t, 1, ua);
        double dprt = dcur + (2.0 * ua[0] - 1.0) * rho * (p->d_max - p->d_min);
        if (dprt < p->d_min) dprt = p->d_min;
        if (dprt > p->d_max) dprt = p->d_max;
        double nprt[3] = {ncur[0] + 2.0 * rho * (2.0 * ua[1] - 1.0), ncur[1] + 2.0 * rho * (2.0 * ua[2] - 1.0),
                          ncur[2] + 2.0 * rho * (2.0 * ua[3] - 1.0)};
        double nn = sqrt(dot3(nprt, nprt));
        nprt[0] /= nn; nprt[1] /= nn; nprt[2] /= nn;
        plane_from(rr, dprt, ncur, cand[n_cand++]);
        plane_from(rr, dcur, nprt, cand[n_cand++]);
        plane_from(rr, dprt, nprt, cand[n_cand++]);
        if (t >= 3) {
            double ub[4], nrnd[3];
            draw4(p, (uint64_t)idx, (uint64_t)t, 2, ub);
            double drnd = p->d_min + ub[0] * (p->d_max - p->d_min);
            normal_from_uniforms(ub[1], ub[2], nrnd);
            plane_from(rr, drnd, ncur, cand[n_cand++]);
            plane_from(rr, dcur, nrnd, cand[n_cand++]);
            plane_from(rr, drnd, nrnd, cand[n_cand++]);
        }
        for (int c = 0; c < n_cand; ++c) {
            if (heuristic) {
                double cc[ORC_MAX_SRC];
                for (int j = 0; j < N; ++j) cc[j] = orc_matching_cost(V, p, x, y, cand[c], j);
                cand_cost[c] = mean_k_lowest(cc, N, p->k);
            } else {
                double acc = 0;
                for (int j = 0; j < N; ++j)
                    if (w[j] > 0.0) acc += w[j] * orc_matching_cost(V, p, x, y, cand[c], j);
                cand_cost[c] = acc / sw;
            }
            if (fabs(cand_cost[c] - cur_cost) < 4 * delta) robust &= ~ORC_ROBUST_REFINE;
            if (cand_cost[c] < cur_cost) {
                cur_cost = cand_cost[c];
                memcpy(cur, cand[c], sizeof(cur));
                chosen = R + 1 + c;
            }
        }
    }

    memcpy(&s->plane[idx * 4], cur, sizeof(cur));
    s->cost[idx] = cur_cost;
    s->S[idx] = S;
    s->v[idx] = v;

    if (dg) {
        for (int r = 0; r <= R; ++r) {
            dg->mfinal[r] = mf[r];
            dg->row_valid[r] = valid[r];
            for (int j = 0; j < N; ++j) dg->M[r][j] = M[r][j];
        }
        for (int r = 0; r < R; ++r) dg->cand_index[r] = cidx[r];
        dg->n_prop = R;
        for (int j = 0; j < N; ++j) dg->w[j] = w[j];
        dg->S = S;
        dg->v = v;
        dg->chosen = chosen;
        dg->n_cand = n_cand;
        for (int c = 0; c < n_cand; ++c) {
            dg->cand_cost[c] = cand_cost[c];
            memcpy(dg->cand_plane[c], cand[c], sizeof(cand[c]));
        }
        dg->robust = robust;
    }
}

void orc_pass(const orc_views *V, const orc_params *p, orc_state *s, int t, int colour,
              const int *order, int n_order, double delta, orc_diag *diag)
{
    int odx[ORC_N_OFFSETS], ody[ORC_N_OFFSETS], oreg[ORC_N_OFFSETS];
    int n_off = p->prop_mode == 1 ? orc_scp_offsets(odx, ody, oreg)
                : p->prop_mode == 2 ? orc_sscp_offsets(odx, ody, oreg) : orc_acp_offsets(odx, ody, oreg);
    long P = (long)V->W * V->H;
    if (order) {
#pragma omp parallel for schedule(dynamic, 16)
        for (long q = 0; q < n_order; ++q) {
            long idx = order[q];
            if (idx < 0 || idx >= P) continue;
            int x = (int)(idx % V->W), y = (int)(idx / V->W);
            if (((x + y) & 1) != colour) continue;
            update_pixel(V, p, s, t, idx, odx, ody, oreg, n_off, delta, diag ? &diag[q] : NULL);
        }
    } else {
#pragma omp parallel for schedule(dynamic, 16)
        for (long idx = 0; idx < P; ++idx) {
            int x = (int)(idx % V->W), y = (int)(idx / V->W);
            if (((x + y) & 1) != colour) continue;
            update_pixel(V, p, s, t, idx, odx, ody, oreg, n_off, delta, NULL);
        }
    }
}

/* schedule (Sec. 3.1, R8): per iteration the red half, then the black half */
void orc_run(const orc_views *V, const orc_params *p, orc_state *s, int iters)
{
    orc_init(V, p, s);
    for (int t = 0; t < iters; ++t) {
        orc_pass(V, p, s, t, 0, NULL, 0, 0.0, NULL);
        orc_pass(V, p, s, t, 1, NULL, 0, 0.0, NULL);
    }
}

void orc_depth_normal(const orc_views *V, const orc_state *s, double *depth, double *normal)
{
    long P = (long)V->W * V->H;
    for (long i = 0; i < P; ++i) {
        int x = (int)(i % V->W), y = (int)(i / V->W);
        depth[i] = depth_at(V, x, y, &s->plane[i * 4]);
        for (int c = 0; c < 3; ++c) normal[i * 3 + c] = s->plane[i * 4 + c];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
