// Depth-map post-processing and fusion (Sec. 3.3, last two paragraphs): the 4x4
// median filter of each depth map and the consistency-check fusion of several
// views' depth and normal maps into one point cloud (the check Gipuma uses,
// with thresholds f_eps on the disparity difference, f_ang on the normal angle
// and f_con consistent views).
//
// Fusion runs one launch triple per reference view, in the order given:
//   fuse_kernel   one lane per pixel of view i: back-project, test every other
//                 view, emit (dense per-pixel point, normal, count) and consume
//                 the witnesses of an emitted pixel in their views' `used` maps;
//   scan_local_kernel   exclusive scan of the 64-pixel block counts within
//                 chunks of 1024 blocks (one workgroup per chunk);
//   scan_chunks_kernel  one workgroup: exclusive scan of the chunk totals,
//                 offset by the points of the views before;
//   scatter_kernel  writes the emitted points in raster order.
// A view's `used` map is written only by the launches of other views, and read
// only by its own, so a launch has no read/write race; the order of the views
// decides which duplicates survive, as in the sequential definition.  Every
// step is deterministic (no atomics), so the cloud is the same on every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "amh_ctx.h"

namespace amh {
namespace {

constexpr int kFuseMaxViews = 128;  // witnesses are recorded in LDS: 4 + 1 bytes x (views - 1) x 64 lanes
constexpr int kGroup = 4;           // views whose gathers are issued together

struct FuseView {
    const float *depth;    // H x W camera z (<= 0 or not finite: no depth)
    const float *normal;   // H x W x 3, camera frame
    unsigned char *used;   // H x W consumed marks
    int W, H;
    float P[12];           // K [R | t], row-major 3 x 4
    float R[9];            // world -> camera rotation, row-major
    float tz;              // t[2]
    float M[9];            // R^T K^-1: pixel (u, v, 1) -> world direction at unit depth
    float C[3];            // camera centre
};

struct FuseArgs {
    const FuseView *views;  // [n]
    int n, i;               // number of views, the reference slot
    const float *fB;        // [n] f_j |C_i - C_j| of this reference
    float f_eps, cos_ang;
    int f_con;
    float4 *pt, *nm;        // dense outputs of view i
    int *cnt;               // -1: no point, else the number of consistent views
    int *block_cnt;         // [nb] point count of each 64-pixel block
    int nb;                 // ceil(P / 64)
};

__device__ __forceinline__ float dot3r(const float *r, float x, float y, float z) {
    return fmaf(r[0], x, fmaf(r[1], y, r[2] * z));
}

__device__ __forceinline__ bool has_depth(float d) { return d > 0.f && d < __builtin_inff(); }

__global__ __launch_bounds__(64) void fuse_kernel(FuseArgs a) {
    extern __shared__ unsigned char fsm[];
    const int lane = threadIdx.x;
    unsigned *wq = reinterpret_cast<unsigned *>(fsm);                          // [n - 1][64] witness pixels
    unsigned char *wj = fsm + sizeof(unsigned) * 64 * (size_t)(a.n - 1);      // [n - 1][64] witness views
    const FuseView &vi = a.views[a.i];
    const long long P = (long long)vi.W * vi.H;
    // XCD-aware order: hardware round-robins workgroups over the 8 XCDs (blockIdx % 8), so XCD x gets the
    // contiguous band of pixel blocks [x per, (x + 1) per) and its L2 sees neighbouring projections
    const int per = (int)(gridDim.x >> 3);
    const int L = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (L >= a.nb) return;  // padding workgroups of the last band (uniform per workgroup)
    const long long p = (long long)L * 64 + lane;
    bool emit = false;
    int cnt = 0;
    float ax = 0.f, ay = 0.f, az = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
    if (p < P) {
        const float d = vi.depth[p];
        if (has_depth(d) && !vi.used[p]) {
            const int y = (int)(p / vi.W), x = (int)(p - (long long)y * vi.W);
            const float xf = (float)x, yf = (float)y;
            const float X = fmaf(d, fmaf(vi.M[0], xf, fmaf(vi.M[1], yf, vi.M[2])), vi.C[0]);
            const float Y = fmaf(d, fmaf(vi.M[3], xf, fmaf(vi.M[4], yf, vi.M[5])), vi.C[1]);
            const float Z = fmaf(d, fmaf(vi.M[6], xf, fmaf(vi.M[7], yf, vi.M[8])), vi.C[2]);
            const float *n0 = vi.normal + 3 * p;
            // world normal R^T n
            const float nx = fmaf(vi.R[0], n0[0], fmaf(vi.R[3], n0[1], vi.R[6] * n0[2]));
            const float ny = fmaf(vi.R[1], n0[0], fmaf(vi.R[4], n0[1], vi.R[7] * n0[2]));
            const float nz = fmaf(vi.R[2], n0[0], fmaf(vi.R[5], n0[1], vi.R[8] * n0[2]));
            ax = X; ay = Y; az = Z;
            bx = nx; by = ny; bz = nz;
            // views in groups of kGroup: every projection of the group first, then all its gathers (independent
            // loads in flight together), then the tests in view order
            for (int j0 = 0; j0 < a.n; j0 += kGroup) {
                float zg[kGroup], ug[kGroup], vg[kGroup], dg[kGroup], mg[kGroup][3];
                long long qg[kGroup];
                bool in[kGroup];
#pragma unroll
                for (int g = 0; g < kGroup; ++g) {
                    const int j = j0 + g;
                    in[g] = false;
                    qg[g] = 0;
                    zg[g] = ug[g] = vg[g] = 0.f;
                    if (j < a.n && j != a.i) {
                        const FuseView &vj = a.views[j];
                        const float z = fmaf(vj.R[6], X, fmaf(vj.R[7], Y, fmaf(vj.R[8], Z, vj.tz)));
                        const float pu = fmaf(vj.P[0], X, fmaf(vj.P[1], Y, fmaf(vj.P[2], Z, vj.P[3])));
                        const float pv = fmaf(vj.P[4], X, fmaf(vj.P[5], Y, fmaf(vj.P[6], Z, vj.P[7])));
                        const float pw = fmaf(vj.P[8], X, fmaf(vj.P[9], Y, fmaf(vj.P[10], Z, vj.P[11])));
                        const float rw = __builtin_amdgcn_rcpf(pw);  // ~1 ulp: 3e-4 px at u ~ 2000
                        const float u = floorf(fmaf(pu, rw, 0.5f)), v = floorf(fmaf(pv, rw, 0.5f));
                        in[g] = z > 0.f && u >= 0.f && u <= (float)(vj.W - 1) && v >= 0.f && v <= (float)(vj.H - 1);
                        if (in[g]) qg[g] = (long long)v * vj.W + (long long)u;
                        zg[g] = z;
                        ug[g] = u;
                        vg[g] = v;
                    }
                }
#pragma unroll
                for (int g = 0; g < kGroup; ++g) {
                    dg[g] = 0.f;
                    mg[g][0] = mg[g][1] = mg[g][2] = 0.f;
                    if (in[g]) {
                        const FuseView &vj = a.views[j0 + g];
                        dg[g] = vj.depth[qg[g]];
                        const float *m = vj.normal + 3 * qg[g];
                        mg[g][0] = m[0];
                        mg[g][1] = m[1];
                        mg[g][2] = m[2];
                    }
                }
#pragma unroll
                for (int g = 0; g < kGroup; ++g) {
                    const int j = j0 + g;
                    const float dj = dg[g];
                    if (!in[g] || !has_depth(dj)) continue;
                    const FuseView &vj = a.views[j];
                    const float disp =
                        a.fB[j] * fabsf(__builtin_amdgcn_rcpf(zg[g]) - __builtin_amdgcn_rcpf(dj));
                    if (!(disp < a.f_eps)) continue;
                    const float mx = fmaf(vj.R[0], mg[g][0], fmaf(vj.R[3], mg[g][1], vj.R[6] * mg[g][2]));
                    const float my = fmaf(vj.R[1], mg[g][0], fmaf(vj.R[4], mg[g][1], vj.R[7] * mg[g][2]));
                    const float mz = fmaf(vj.R[2], mg[g][0], fmaf(vj.R[5], mg[g][1], vj.R[8] * mg[g][2]));
                    if (!(fmaf(nx, mx, fmaf(ny, my, nz * mz)) > a.cos_ang)) continue;
                    ax += fmaf(dj, dot3r(vj.M, ug[g], vg[g], 1.f), vj.C[0]);
                    ay += fmaf(dj, dot3r(vj.M + 3, ug[g], vg[g], 1.f), vj.C[1]);
                    az += fmaf(dj, dot3r(vj.M + 6, ug[g], vg[g], 1.f), vj.C[2]);
                    bx += mx; by += my; bz += mz;
                    wq[cnt * 64 + lane] = (unsigned)qg[g];
                    wj[cnt * 64 + lane] = (unsigned char)j;
                    ++cnt;
                }
            }
            emit = cnt >= a.f_con;
        }
    }
    if (p < P) {
        if (emit) {
            const float inv = 1.f / (float)(cnt + 1);
            const float nn = 1.f / sqrtf(fmaf(bx, bx, fmaf(by, by, bz * bz)));
            a.pt[p] = make_float4(ax * inv, ay * inv, az * inv, 0.f);
            a.nm[p] = make_float4(bx * nn, by * nn, bz * nn, 0.f);
            for (int k = 0; k < cnt; ++k) {
                const FuseView &vj = a.views[wj[k * 64 + lane]];
                vj.used[wq[k * 64 + lane]] = 1;
            }
        }
        a.cnt[p] = emit ? cnt : -1;
    }
    const unsigned long long b = __ballot(emit);
    if (lane == 0) a.block_cnt[L] = __popcll(b);
}

// Inclusive scan over a workgroup of 1024 threads; returns this thread's inclusive prefix and the total.
__device__ __forceinline__ long long block_scan_1024(long long v, long long *wsum, long long &total) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        long long s = lane < 16 ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const long long u = __shfl_up(s, o, 64);
            if (lane >= o) s += u;
        }
        if (lane < 16) wsum[lane] = s;  // inclusive prefix of the wave totals
    }
    __syncthreads();
    total = wsum[15];
    const long long r = v + (w > 0 ? wsum[w - 1] : 0);
    __syncthreads();  // wsum is reused by the caller's next scan
    return r;
}

// Block counts -> exclusive offsets within chunks of 1024 blocks; chunk totals.
__global__ __launch_bounds__(1024) void scan_local_kernel(const int *block_cnt, int nb, int *local_off,
                                                          long long *chunk_sum) {
    __shared__ long long wsum[16];
    const int b = blockIdx.x * 1024 + threadIdx.x;
    const long long v = b < nb ? block_cnt[b] : 0;
    long long total;
    const long long inc = block_scan_1024(v, wsum, total);
    if (b < nb) local_off[b] = (int)(inc - v);
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = total;
}

// Chunk totals -> exclusive chunk offsets starting at *total; *total += the sum.
__global__ __launch_bounds__(1024) void scan_chunks_kernel(const long long *chunk_sum, int nc, long long *chunk_off,
                                                           long long *total) {
    __shared__ long long wsum[16];
    long long carry = *total;
    for (int c0 = 0; c0 < nc; c0 += 1024) {
        const int c = c0 + (int)threadIdx.x;
        const long long v = c < nc ? chunk_sum[c] : 0;
        long long tot;
        const long long inc = block_scan_1024(v, wsum, tot);
        if (c < nc) chunk_off[c] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(64) void scatter_kernel(const float4 *pt, const float4 *nm, const int *cnt,
                                                     const int *local_off, const long long *chunk_off, long long P,
                                                     int slot, float *points, float *normals, int *origin,
                                                     long long cap) {
    const int lane = threadIdx.x;
    const long long p = (long long)blockIdx.x * 64 + lane;
    const bool has = p < P && cnt[p] >= 0;
    const unsigned long long b = __ballot(has);
    if (!has) return;
    const long long pos = chunk_off[blockIdx.x >> 10] + local_off[blockIdx.x] + __popcll(b & ((1ull << lane) - 1ull));
    if (pos >= cap) return;
    const float4 x = pt[p];
    points[3 * pos] = x.x;
    points[3 * pos + 1] = x.y;
    points[3 * pos + 2] = x.z;
    if (normals) {
        const float4 n = nm[p];
        normals[3 * pos] = n.x;
        normals[3 * pos + 1] = n.y;
        normals[3 * pos + 2] = n.z;
    }
    if (origin) {
        origin[3 * pos] = slot;
        origin[3 * pos + 1] = (int)p;
        origin[3 * pos + 2] = cnt[p];
    }
}

__global__ void fill_u8_kernel(unsigned char *p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void zero_i64_kernel(long long *p) {
    if (threadIdx.x == 0) *p = 0;
}

// 4x4 median: window columns x-1..x+2, rows y-1..y+2 clipped to the image, NaN skipped; sorted with a
// bitonic network (absent values are +inf and sort last); even counts average the two middle values.
__global__ __launch_bounds__(256) void median4_kernel(const float *__restrict__ src, float *__restrict__ dst, int W,
                                                      int H) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    float v[16];
    int n = 0;
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 4; ++dx) {
            const int xx = x + dx - 1, yy = y + dy - 1;
            float s = __builtin_inff();
            if (xx >= 0 && xx < W && yy >= 0 && yy < H) {
                const float r = src[(size_t)yy * W + xx];
                if (!isnan(r)) {
                    s = r;
                    ++n;
                }
            }
            v[dy * 4 + dx] = s;
        }
    }
#pragma unroll
    for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const float lo = fminf(v[i], v[l]), hi = fmaxf(v[i], v[l]);
                    const bool up = (i & k) == 0;
                    v[i] = up ? lo : hi;
                    v[l] = up ? hi : lo;
                }
            }
        }
    }
    const int h = n >> 1;
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k == h - 1) a = v[k];
        if (k == h) b = v[k];
    }
    dst[(size_t)y * W + x] = n == 0 ? __builtin_nanf("") : ((n & 1) ? b : 0.5f * (a + b));
}

#define AMH_LAUNCH_F(...)                \
    do {                                 \
        (void)hipGetLastError();         \
        hipLaunchKernelGGL(__VA_ARGS__); \
    } while (0)

}  // namespace

void free_fusion(amh_ctx *c) {
    if (c->fuse_ws) (void)hipFree(c->fuse_ws);
    c->fuse_ws = nullptr;
    c->fuse_ws_cap = 0;
    for (auto e : c->fuse_ev) (void)hipEventDestroy(e);
    c->fuse_ev.clear();
}

}  // namespace amh

extern "C" {

amh_status amh_fusion_params_default(amh_fusion_params *out) {
    if (!out) return AMH_E_INVALID_ARG;
    out->f_eps = 0.3f;
    out->f_ang_deg = 30.f;
    out->f_con = 2;
    return AMH_OK;
}

amh_status amh_median_filter4(amh_ctx *c, const float *src, float *dst, int width, int height) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!src || !dst) return fail(c, AMH_E_INVALID_ARG, "src and dst are required");
    if (src == dst) return fail(c, AMH_E_INVALID_ARG, "the median filter does not run in place (src == dst)");
    if (width < 1 || height < 1 || (long long)width * height > (1ll << 31) - 1)
        return fail(c, AMH_E_INVALID_ARG, "need 1 <= width, height and width * height < 2^31");
    dim3 grid((width + 63) / 64, (height + 3) / 4);
    AMH_LAUNCH_F(median4_kernel, grid, dim3(256), 0, c->stream, src, dst, width, height);
    HIPCHK(c, hipGetLastError());
    return AMH_OK;
}

amh_status amh_fuse(amh_ctx *c, int n_views, const int *views, const float *const *depth, const float *const *normal,
                    const amh_fusion_params *fp, float *points, float *point_normals, int32_t *origin,
                    int64_t capacity, int64_t *n_points) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!views || !depth || !normal || !fp || !n_points)
        return fail(c, AMH_E_INVALID_ARG, "views, depth, normal, params and n_points are required");
    if (n_views < 1 || n_views > kFuseMaxViews) return fail(c, AMH_E_INVALID_ARG, "need 1 <= n_views <= %d", kFuseMaxViews);
    if (!(fp->f_eps > 0.f) || !std::isfinite(fp->f_eps) || !(fp->f_ang_deg > 0.f && fp->f_ang_deg <= 180.f) ||
        fp->f_con < 0)
        return fail(c, AMH_E_INVALID_ARG, "need f_eps > 0 finite, 0 < f_ang_deg <= 180, f_con >= 0");
    if (capacity < 0 || (capacity > 0 && !points))
        return fail(c, AMH_E_INVALID_ARG, "capacity >= 0, and points is required when capacity > 0");
    const int nv = (int)c->views.size();
    long long maxP = 0, sumP = 0;
    for (int k = 0; k < n_views; ++k) {
        if (views[k] < 0 || views[k] >= nv) return fail(c, AMH_E_INVALID_ARG, "view %d is not registered", views[k]);
        if (!depth[k] || !normal[k]) return fail(c, AMH_E_INVALID_ARG, "depth[%d] and normal[%d] are required", k, k);
        const View &v = c->views[views[k]];
        const long long P = (long long)v.W * v.H;
        if (P > (1ll << 31) - 1) return fail(c, AMH_E_UNSUPPORTED, "view %d has 2^31 pixels or more", views[k]);
        maxP = std::max(maxP, P);
        sumP += P;
    }
    const long long maxB = (maxP + 63) / 64;
    const long long maxC = (maxB + 1023) / 1024;
    // workspace: used marks, dense point / normal / count of one view, block offsets, the view table,
    // the baselines and the running total
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_used = 0;
    const size_t o_pt = o_used + al((size_t)sumP);
    const size_t o_nm = o_pt + al((size_t)maxP * 16);
    const size_t o_cnt = o_nm + al((size_t)maxP * 16);
    const size_t o_blk = o_cnt + al((size_t)maxP * 4);
    const size_t o_loc = o_blk + al((size_t)maxB * 4);
    const size_t o_csum = o_loc + al((size_t)maxB * 4);
    const size_t o_coff = o_csum + al((size_t)maxC * 8);
    const size_t o_views = o_coff + al((size_t)maxC * 8);
    const size_t o_fb = o_views + al(sizeof(FuseView) * n_views);
    const size_t o_tot = o_fb + al(sizeof(float) * n_views * n_views);
    const size_t need = o_tot + 256;
    if (need > c->fuse_ws_cap) {
        free_fusion(c);
        amh_status s = dalloc(c, &c->fuse_ws, need);
        if (s != AMH_OK) return s;
        c->fuse_ws_cap = need;
    }
    unsigned char *ws = static_cast<unsigned char *>(c->fuse_ws);
    // view table (host, double precision, then float)
    std::vector<FuseView> hv(n_views);
    std::vector<double> cen(3 * n_views);
    std::vector<double> fx(n_views);
    size_t used_off = 0;
    for (int k = 0; k < n_views; ++k) {
        const View &v = c->views[views[k]];
        FuseView &f = hv[k];
        f.depth = depth[k];
        f.normal = normal[k];
        f.used = ws + o_used + used_off;
        used_off += (size_t)v.W * v.H;
        f.W = v.W;
        f.H = v.H;
        const double *K = v.K, *R = v.R, *t = v.t;
        for (int r = 0; r < 3; ++r) {
            for (int q = 0; q < 3; ++q) {
                double s = 0;
                for (int m = 0; m < 3; ++m) s += K[3 * r + m] * R[3 * m + q];
                f.P[4 * r + q] = (float)s;
            }
            double s = 0;
            for (int m = 0; m < 3; ++m) s += K[3 * r + m] * t[m];
            f.P[4 * r + 3] = (float)s;
        }
        for (int q = 0; q < 9; ++q) f.R[q] = (float)R[q];
        f.tz = (float)t[2];
        // K^-1 of an upper-triangular K
        double Ki[9] = {0};
        Ki[0] = 1.0 / K[0];
        Ki[1] = -K[1] / (K[0] * K[4]);
        Ki[2] = (K[1] * K[5] - K[2] * K[4]) / (K[0] * K[4] * K[8]);
        Ki[4] = 1.0 / K[4];
        Ki[5] = -K[5] / (K[4] * K[8]);
        Ki[8] = 1.0 / K[8];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                double s = 0;
                for (int m = 0; m < 3; ++m) s += R[3 * m + r] * Ki[3 * m + q];  // (R^T Ki)[r][q]
                f.M[3 * r + q] = (float)s;
            }
        for (int r = 0; r < 3; ++r) {
            double s = 0;
            for (int m = 0; m < 3; ++m) s -= R[3 * m + r] * t[m];
            cen[3 * k + r] = s;
            f.C[r] = (float)s;
        }
        fx[k] = K[0] / K[8];
    }
    std::vector<float> fB((size_t)n_views * n_views);
    for (int i = 0; i < n_views; ++i)
        for (int j = 0; j < n_views; ++j) {
            const double dx = cen[3 * i] - cen[3 * j], dy = cen[3 * i + 1] - cen[3 * j + 1],
                         dz = cen[3 * i + 2] - cen[3 * j + 2];
            fB[(size_t)i * n_views + j] = (float)(fx[j] * std::sqrt(dx * dx + dy * dy + dz * dz));
        }
    FuseView *d_views = reinterpret_cast<FuseView *>(ws + o_views);
    float *d_fb = reinterpret_cast<float *>(ws + o_fb);
    long long *d_total = reinterpret_cast<long long *>(ws + o_tot);
    int *d_blk = reinterpret_cast<int *>(ws + o_blk);
    int *d_loc = reinterpret_cast<int *>(ws + o_loc);
    long long *d_csum = reinterpret_cast<long long *>(ws + o_csum);
    long long *d_coff = reinterpret_cast<long long *>(ws + o_coff);
    float4 *d_pt = reinterpret_cast<float4 *>(ws + o_pt);
    float4 *d_nm = reinterpret_cast<float4 *>(ws + o_nm);
    int *d_cnt = reinterpret_cast<int *>(ws + o_cnt);
    HIPCHK(c, hipMemcpyAsync(d_views, hv.data(), sizeof(FuseView) * n_views, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_fb, fB.data(), sizeof(float) * fB.size(), hipMemcpyHostToDevice, c->stream));
    AMH_LAUNCH_F(fill_u8_kernel, dim3(1024), dim3(256), 0, c->stream, ws + o_used, sumP);
    HIPCHK(c, hipGetLastError());
    AMH_LAUNCH_F(zero_i64_kernel, dim3(1), dim3(64), 0, c->stream, d_total);
    HIPCHK(c, hipGetLastError());
    const float cos_ang = (float)std::cos((double)fp->f_ang_deg * 3.14159265358979323846 / 180.0);
    const bool timed = c->p.timing != 0;
    c->fuse_ms = 0.f;
    c->fuse_n = 0;
    while (timed && c->fuse_ev.size() < 2 * (size_t)n_views) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->fuse_ev.push_back(e);
    }
    const size_t lds = (size_t)(n_views - 1) * 64 * (sizeof(unsigned) + 1);
    for (int i = 0; i < n_views; ++i) {
        const long long P = (long long)hv[i].W * hv[i].H;
        const int nb = (int)((P + 63) / 64);
        FuseArgs a;
        a.views = d_views;
        a.n = n_views;
        a.i = i;
        a.fB = d_fb + (size_t)i * n_views;
        a.f_eps = fp->f_eps;
        a.cos_ang = cos_ang;
        a.f_con = fp->f_con;
        a.pt = d_pt;
        a.nm = d_nm;
        a.cnt = d_cnt;
        a.block_cnt = d_blk;
        a.nb = nb;
        if (timed) HIPCHK(c, hipEventRecord(c->fuse_ev[2 * i], c->stream));
        AMH_LAUNCH_F(fuse_kernel, dim3(((nb + 7) / 8) * 8), dim3(64), lds, c->stream, a);
        HIPCHK(c, hipGetLastError());
        if (timed) HIPCHK(c, hipEventRecord(c->fuse_ev[2 * i + 1], c->stream));
        const int nc = (nb + 1023) / 1024;
        AMH_LAUNCH_F(scan_local_kernel, dim3(nc), dim3(1024), 0, c->stream, d_blk, nb, d_loc, d_csum);
        HIPCHK(c, hipGetLastError());
        AMH_LAUNCH_F(scan_chunks_kernel, dim3(1), dim3(1024), 0, c->stream, d_csum, nc, d_coff, d_total);
        HIPCHK(c, hipGetLastError());
        AMH_LAUNCH_F(scatter_kernel, dim3(nb), dim3(64), 0, c->stream, d_pt, d_nm, d_cnt, d_loc, d_coff, P, i,
                     points, point_normals, origin, (long long)capacity);
        HIPCHK(c, hipGetLastError());
    }
    long long total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, d_total, sizeof(total), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *n_points = total;
    if (timed) {
        for (int i = 0; i < n_views; ++i) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->fuse_ev[2 * i], c->fuse_ev[2 * i + 1]));
            c->fuse_ms += ms;
        }
        c->fuse_n = n_views;
    }
    return AMH_OK;
}

}  // extern "C"
