/*
 * Drives every entry point of the CPU oracle on a small synthetic scene, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py compiles and runs it).  Exit status 0 when
 * every call returned and its outputs are finite and in range.
 *
 * Scene: a reference and three sources with the reference camera's intrinsics,
 * translated along x and y; textures are a fixed integer hash, so no library
 * random generator is involved.  Sizes are odd (ragged tiles), and the runs
 * cover every mode: joint view selection, the static objective, heuristic
 * selection, symmetric propagation (fast and standard), squared weights, no self row, the
 * conditioning probes (every level), refinement before and after t = 3, and per-pixel
 * diagnostics over an explicit pixel order.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/amh_oracle.h"

static float texel(uint32_t x, uint32_t y, uint32_t salt)
{
    uint32_t h = x * 0x9E3779B1u ^ (y + 0x7F4A7C15u) * 0x85EBCA77u ^ salt * 0xC2B2AE3Du;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (float)(h % 256u);
}

static int check_state(const orc_state *s, long P, int n_src)
{
    for (long i = 0; i < P; ++i) {
        for (int c = 0; c < 4; ++c)
            if (!isfinite(s->plane[4 * i + c])) return 1;
        if (!(s->cost[i] >= 0.0 && s->cost[i] <= 2.0)) return 2;
        if (s->v[i] < -1 || s->v[i] >= n_src) return 3;
        if (n_src < 32 && (s->S[i] >> n_src) != 0u) return 4;
    }
    return 0;
}

int main(void)
{
    enum { W = 37, H = 29, NS = 3 };
    const long P = (long)W * H;
    float *img[NS + 1];
    for (int k = 0; k <= NS; ++k) {
        img[k] = malloc(sizeof(float) * P);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) img[k][(long)y * W + x] = texel((uint32_t)(x + 2 * k), (uint32_t)y, 7u);
    }
    orc_views V;
    memset(&V, 0, sizeof V);
    V.W = W;
    V.H = H;
    V.n_src = NS;
    V.ref = img[0];
    const double K[9] = {40.0, 0.0, (W - 1) / 2.0, 0.0, 40.0, (H - 1) / 2.0, 0.0, 0.0, 1.0};
    const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(V.Kref, K, sizeof K);
    memcpy(V.Rref, I, sizeof I);
    for (int j = 0; j < NS; ++j) {
        V.src[j] = img[j + 1];
        V.srcW[j] = W;
        V.srcH[j] = H;
        memcpy(V.Ksrc[j], K, sizeof K);
        memcpy(V.Rsrc[j], I, sizeof I);
        V.tsrc[j][0] = -0.05 * (j + 1);
        V.tsrc[j][1] = j == 2 ? 0.03 : 0.0;
    }
    orc_state s;
    s.plane = malloc(sizeof(double) * 4 * P);
    s.cost = malloc(sizeof(double) * P);
    s.S = malloc(sizeof(uint32_t) * P);
    s.v = malloc(sizeof(int32_t) * P);
    int *order = malloc(sizeof(int) * P);
    orc_diag *dg = malloc(sizeof(orc_diag) * P);
    int rc = 0;
    for (int mode = 0; mode < 11 && rc == 0; ++mode) {
        orc_params p;
        memset(&p, 0, sizeof p);
        p.refine = 1;
        p.include_self = mode != 3;
        p.d_min = 2.0;
        p.d_max = 6.0;
        p.sigma_color = 3.0;
        p.sigma_spatial = 30.0;
        p.tau_mc_init = 0.8;
        p.alpha = 90.0;
        p.beta = 0.3;
        p.tau_up = 1.2;
        p.n1 = 2;
        p.n2 = 3;
        p.k = mode == 4 ? 1 : 4;
        p.seed = 11u + (uint64_t)mode;
        p.view_mode = mode == 1 ? 1 : (mode == 2 ? 2 : 0);
        p.prop_mode = mode == 5 ? 1 : (mode == 10 ? 2 : 0);
        p.bilateral_sq = mode == 6;
        p.sample_f32 = mode == 7 ? 1 : (mode == 8 ? 2 : (mode == 9 ? 3 : 0));
        p.cost_noise = mode == 7 ? 2e-4 : 0.0;
        orc_run(&V, &p, &s, 2);
        if ((rc = check_state(&s, P, NS)) != 0) break;
        /* diagnostics over an explicit order (reversed raster, with out-of-range entries) at t = 1 and 3 */
        for (int t = 1; t <= 3 && rc == 0; t += 2) {
            for (int colour = 0; colour < 2; ++colour) {
                int n = 0;
                for (long i = P - 1; i >= 0; --i) order[n++] = (int)i;
                order[0] = -5;
                order[1] = (int)P + 3;
                orc_pass(&V, &p, &s, t, colour, order, n, 1e-5, dg);
                rc = check_state(&s, P, NS);
            }
        }
        double d[W * H], nrm[3 * W * H];
        orc_depth_normal(&V, &s, d, nrm);
        for (long i = 0; i < P && rc == 0; ++i)
            if (!(d[i] > 0.0) || !isfinite(nrm[3 * i])) rc = 10;
        if (rc) fprintf(stderr, "mode %d: check %d failed\n", mode, rc);
    }
    /* the remaining public functions */
    int dx[ORC_N_OFFSETS], dy[ORC_N_OFFSETS], reg[ORC_N_OFFSETS];
    if (orc_acp_offsets(dx, dy, reg) != ORC_N_OFFSETS || orc_scp_offsets(dx, dy, reg) != 8 ||
        orc_sscp_offsets(dx, dy, reg) != 20)
        rc = 20;
    double M[8 * NS], w[NS];
    int rv[8] = {1, 1, 1, 1, 1, 1, 0, 1};
    for (int i = 0; i < 8 * NS; ++i) M[i] = (i % 5) * 0.3;
    uint32_t So;
    int vo;
    orc_params p0;
    memset(&p0, 0, sizeof p0);
    p0.tau_mc_init = 0.8;
    p0.alpha = 90.0;
    p0.beta = 0.3;
    p0.tau_up = 1.2;
    p0.n1 = 2;
    p0.n2 = 3;
    p0.k = 4;
    orc_view_selection(&p0, 2, M, rv, NS, 1u, 0, &So, &vo, w);
    for (int j = 0; j < NS; ++j)
        if (!(w[j] >= 0.0)) rc = 21;
    orc_set_num_threads(1);
    if (orc_num_threads() < 1) rc = 22;
    for (int k = 0; k <= NS; ++k) free(img[k]);
    free(s.plane);
    free(s.cost);
    free(s.S);
    free(s.v);
    free(order);
    free(dg);
    printf("oracle sanitizer run: %s\n", rc ? "FAILED" : "ok");
    return rc;
}
