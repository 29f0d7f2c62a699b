// gfx950 kernels of the checkerboard PatchMatch pass (Xu & Tao, arXiv 1805.07920).
//
// Work mapping of the pass (Sec. 3.1-3.3): a wave64 holds 7 pixels of one
// colour on one image row, 9 lanes each.  Lane r < 8 owns the hypothesis
// propagated from asymmetric region r, lane 8 the pixel's own plane; the
// 64th lane idles.  All lanes of a wave warp into the same source view at the
// same time, so their bilinear gathers hit neighbouring texels.  A workgroup
// (4 waves) covers a tile of 4 rows x 7 same-colour pixels; its reference
// window (tile + 5 px halo) is staged once in LDS.  The 9 x N cost matrix of a
// pixel lives in LDS, one column per view; view selection is split over the
// 9 lanes of the pixel and the final argmin is a 9-lane reduction.  MFMA is
// not used: the work is per-sample gathers and scalar arithmetic, bounded by
// the vector ALU.
#include <hip/hip_fp16.h>

#include <algorithm>
#include <hip/hip_runtime.h>

#include "amh_bf16.h"
#include "amh_internal.h"

// Minimum waves per SIMD the kernels are compiled for (a register budget of
// 512 / waves VGPRs).  The single-image and batched half-passes are held to 4
// waves per SIMD (128 VGPRs), which they fit without spilling; the ablation
// build gets the budget of 2 waves and settles near 125 VGPRs by itself; the
// initialisation kernels, which hold half a window block per lane, fit 3
// waves (at 4 they spill inside the source loop).
#ifndef AMH_PASS_WAVES_PER_EU
#define AMH_PASS_WAVES_PER_EU 4
#endif
#ifndef AMH_BATCH_WAVES_PER_EU
#define AMH_BATCH_WAVES_PER_EU 2
#endif
#ifndef AMH_INIT_WAVES_PER_EU
#define AMH_INIT_WAVES_PER_EU 3
#endif

namespace amh {

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Key (seed, 0),
// counter (pixel, iteration, purpose, 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint64_t pix, uint64_t it, uint64_t purpose, uint64_t seed, float u[4]) {
    uint64_t c0 = pix, c1 = it, c2 = purpose, c3 = 0;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        uint64_t h0 = __umul64hi(m0, c0), l0 = m0 * c0;
        uint64_t h1 = __umul64hi(m1, c2), l1 = m1 * c2;
        uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0; c1 = l1; c2 = n2; c3 = l0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    // top 24 bits -> [0, 1), exact in float
    u[0] = (float)(uint32_t)(c0 >> 40) * 0x1p-24f;
    u[1] = (float)(uint32_t)(c1 >> 40) * 0x1p-24f;
    u[2] = (float)(uint32_t)(c2 >> 40) * 0x1p-24f;
    u[3] = (float)(uint32_t)(c3 >> 40) * 0x1p-24f;
}

// ---------------------------------------------------------------------------
// Asymmetric checkerboard propagation regions (Sec. 3.1, Fig. 2(d)).
// Regions 0-3: near V-shaped wedges (7 candidates) up/down/left/right,
// regions 4-7: far axial strips (11 candidates, odd distances 3..23).
// Candidate e of the "up" wedge sits at level l = (e + 1) / 2 (0..3) beside
// the axis, alternating left/right; far candidates step by 2 px.
// Every offset has odd |dx| + |dy|, i.e. the other colour.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int region_size(int r) { return r < 4 ? 7 : 11; }

__device__ __forceinline__ void region_offset(int r, int e, int &dx, int &dy) {
    int ux, uy;
    if (r < 4) {
        int lvl = (e + 1) >> 1;
        int side = (e & 1) ? -1 : 1;
        ux = side * lvl;
        uy = -(lvl + 1);
    } else {
        ux = 0;
        uy = -(3 + 2 * e);
    }
    switch (r & 3) {
        case 0: dx = ux; dy = uy; break;     // up
        case 1: dx = ux; dy = -uy; break;    // down
        case 2: dx = uy; dy = ux; break;     // left
        default: dx = -uy; dy = ux; break;   // right
    }
}

// ---------------------------------------------------------------------------
// Texel columns: entry (y0 + 1 + P, x0 + 1 + P) of a (H+1+2P) x (W+2+2P)
// array (P = kQuadPad) holds the vertical texel pair a = (x0, y0),
// c = (x0, y0 + 1), x0 in [-1-P, W+P], y0 in [-1-P, H-1+P], indices clamped to
// the image.  Two neighbouring entries are the bilinear footprint with top-left
// texel (x0, y0) -- a, c and b = (x0+1, y0), d = (x0+1, y0+1) -- so one 16-byte
// (8-byte) load at an 8-byte (4-byte) aligned address serves a sample, and a
// sample up to P texels outside the image reads what clamping its indices would
// read.  At 8 (4) bytes per texel the layout is half the size of one holding
// the four texels per texel, which halves the lines a window row touches and
// the footprint the caches must hold where the hypotheses are random.
//   float32: (a, c - a), the difference rounded once from its exact value; a
//            sample is L + fx (R - L) with L = a + fy (c - a), R = b + fy (d - b);
//   float16: the texels (a, c) themselves (differences would not be exact in
//            half precision).
// Offsets are 32-bit byte offsets from a wave-uniform base (global loads with
// a scalar base address).
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(1))) unsigned char gbyte;

// The library's buffers are global memory; a pointer read from a table (batched launches) reaches the
// kernels as a generic one, so state and reference accesses name the global address space explicitly
// (global instead of flat instructions).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *glob(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
typedef float gf4 __attribute__((ext_vector_type(4)));

// planes (float4) through the global address space, as the clang vector type
__device__ __forceinline__ float4 load_plane(const float4 *base, size_t i) {
    const gf4 v = ((const __attribute__((address_space(1))) gf4 *)base)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store_plane(float4 *base, size_t i, float4 p) {
    gf4 v;
    v.x = p.x;
    v.y = p.y;
    v.z = p.z;
    v.w = p.w;
    ((__attribute__((address_space(1))) gf4 *)base)[i] = v;
}
typedef _Float16 gh4 __attribute__((ext_vector_type(4)));

template <int HALF>
struct QuadT {
    typedef gf4 type;
};
template <>
struct QuadT<1> {
    typedef gh4 type;
};

// the footprint (two neighbouring entries) at half its natural alignment
typedef float gf4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef _Float16 gh4a4 __attribute__((ext_vector_type(4), aligned(4)));
template <int HALF>
struct QuadLd {
    typedef gf4a8 type;
};
template <>
struct QuadLd<1> {
    typedef gh4a4 type;
};

template <int HALF>
__device__ __forceinline__ typename QuadT<HALF>::type load_quad(const void *base, uint32_t off) {
    return *reinterpret_cast<const __attribute__((address_space(1))) typename QuadLd<HALF>::type *>(
        (gbyte *)base + off);
}

// q = (a, c - a, b, d - b)
__device__ __forceinline__ float eval_quad_f32(gf4 q, float fx, float fy) {
    const float l = fmaf(fy, q.y, q.x), r = fmaf(fy, q.w, q.z);
    return fmaf(fx, r - l, l);
}

// q = (a, c, b, d)
__device__ __forceinline__ float eval_quad_f16(gh4 q, float fx, float fy) {
    // a + fx (b - a) as fma(b, fx, fma(-a, fx, a)): the halves enter mixed-precision FMAs directly
    // (exact conversion inside the instruction), which saves the separate conversions and differences
    const float a = (float)q.x, c = (float)q.y, b = (float)q.z, d = (float)q.w;
    const float top = fmaf(b, fx, fmaf(-a, fx, a));
    const float bot = fmaf(d, fx, fmaf(-c, fx, c));
    return fmaf(fy, bot - top, top);
}

template <int HALF>
__device__ __forceinline__ float eval_quad(typename QuadT<HALF>::type q, float fx, float fy);
template <>
__device__ __forceinline__ float eval_quad<0>(gf4 q, float fx, float fy) { return eval_quad_f32(q, fx, fy); }
template <>
__device__ __forceinline__ float eval_quad<1>(gh4 q, float fx, float fy) { return eval_quad_f16(q, fx, fy); }

// floor(x) converted to int in one instruction, and a 3-operand clamp
__device__ __forceinline__ int cvt_floor(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ int med3i(int x, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// Warps the 6 samples of window row vf (pixel offset -5..5) into the source and
// issues their texel loads.  The homogeneous source position of window offset
// (u, v) is (N0 + u Pu + v Pv) relative to the texel (ix, iy); texel indices
// are clamped to the image (-1..W-1 in absolute terms, the quad layout holds
// the clamped footprint).  CLAMP = false: the caller has shown that every
// index is already inside that range, so the clamp would change nothing.
template <int HALF, bool CLAMP>
__device__ __forceinline__ void issue_row(const void *quads, float vf, float N0x, float N0y, float Z0, float pux,
                                          float puy, float puz, float pvx, float pvy, float pvz, int xlo, int xhi,
                                          int ylo, int yhi, int row_bytes, int base,
                                          typename QuadT<HALF>::type (&qd)[6], float (&fxs)[6], float (&fys)[6]) {
    constexpr int kEntry = HALF ? 4 : 8;
    const float rx = fmaf(vf, pvx, N0x), ry = fmaf(vf, pvy, N0y), rzz = fmaf(vf, pvz, Z0);
#pragma unroll
    for (int su = 0; su < 6; ++su) {
        const float uf = -5.f + 2.f * su;
        const float nx = fmaf(uf, pux, rx), ny = fmaf(uf, puy, ry), nz = fmaf(uf, puz, rzz);
        const float r = __builtin_amdgcn_rcpf(nz);
        const float dx = nx * r, dy = ny * r;
        const int xr = CLAMP ? med3i(cvt_floor(dx), xlo, xhi) : cvt_floor(dx);
        const int yr = CLAMP ? med3i(cvt_floor(dy), ylo, yhi) : cvt_floor(dy);
        fxs[su] = __builtin_amdgcn_fractf(dx);
        fys[su] = __builtin_amdgcn_fractf(dy);
        // modulo-2^32 arithmetic; the true offset is in [0, (W+2+2P)(H+1+2P) * entry) <= 2^32
        const uint32_t off = (uint32_t)__mul24(yr, row_bytes) + (uint32_t)base + (uint32_t)xr * kEntry;
        qd[su] = load_quad<HALF>(quads, off);
    }
}

// ---------------------------------------------------------------------------
// Reference window of a pixel (Sec. 3.3): 36 samples at offsets
// {-5,-3,-1,1,3,5}^2, bilateral weights w = exp(-|a - a_c| / (2 sc^2)
// - dist / (2 sx^2)) from the reference patch.  Stored per sample as
// (w, w * (a - mean_w a)) so that the source loop only accumulates moments of
// the source samples.  Returns 1/sum(w) and the reference's weighted variance.
// ---------------------------------------------------------------------------
struct WinStats {
    float invW, var_a;
};

// A pixel's window block in LDS: 36 x (w, w (a - mean)) followed by 6 per-row
// constants (1 / W_r, W_r / W_<=r, W_<r W_r / W_<=r, A_r) with W_r the row's
// weight sum and A_r its sum of w (a - mean); they let the source moments be
// formed row by row and merged exactly (see ncc_cost).
constexpr int kWinStride = 48;  // float2 units: 36 + 6 float4

// Computes a pixel's window block and hands each entry to the sink: sink.sample(s, (w, w (a - mean))) for the
// 36 samples, sink.row(r, constants) for the 6 rows.
template <typename Reader, typename Sink>
__device__ __forceinline__ WinStats build_window_to(const Reader &rd, const MethodDev &m, Sink &sink) {
    // every operation rounded as written: the kernels that build a pixel's block must agree bit for bit, and
    // a contraction the compiler may or may not make in each of them would break that
#pragma clang fp contract(off)
    float a[36];
    const float ac = rd(0, 0);
    float sw = 0.f, swa = 0.f;
    float w[36];
    // exponents of the weights: unsquared colour difference and distance as printed (Eq. 8), or the
    // squared form; the weights are scaled by exp(min exponent), a common factor that cancels in the
    // NCC, so the largest is 1 and the sum never underflows
    float emin = __builtin_inff();
#pragma unroll
    for (int s = 0; s < 36; ++s) {
        const int du = -5 + 2 * (s % 6), dv = -5 + 2 * (s / 6);
        a[s] = rd(du, dv);
        const float d2 = (float)(du * du + dv * dv), dc = fabsf(a[s] - ac);
        const float dist = m.bil_sq ? d2 : __builtin_sqrtf(d2);
        const float col = m.bil_sq ? dc * dc : dc;
        w[s] = fmaf(col, m.inv_2sc2, dist * m.inv_2sx2);
        emin = fminf(emin, w[s]);
    }
#pragma unroll
    for (int s = 0; s < 36; ++s) {
        w[s] = __expf(emin - w[s]);
        sw += w[s];
        swa = fmaf(w[s], a[s], swa);
    }
    const float invW = 1.f / sw;
    const float mean = swa * invW;
    float saa = 0.f;
    float wcum = 0.f;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        float wr = 0.f, ar = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int s = r * 6 + k;
            const float ap = a[s] - mean;
            const float wap = w[s] * ap;
            saa = fmaf(wap, ap, saa);
            wr += w[s];
            ar += wap;
            sink.sample(s, make_float2(w[s], wap));
        }
        const float wprev = wcum;
        wcum += wr;
        // a row whose weights all underflow adds nothing (its constants are 0)
        sink.row(r, wr > 0.f ? make_float4(1.f / wr, wr / wcum, wprev * wr / wcum, ar) : make_float4(0.f, 0.f, 0.f, 0.f));
    }
    WinStats ws;
    ws.invW = invW;
    ws.var_a = saa * invW;
    return ws;
}

// The window block of one pixel in its lane's registers: the 36 sample entries and 6 row constants.
struct RegWin {
    float2 smp[36];
    float4 rc[6];
};
struct RegWinSink {
    RegWin *win;
    __device__ __forceinline__ void sample(int s, float2 v) const { win->smp[s] = v; }
    __device__ __forceinline__ void row(int r, float4 v) const { win->rc[r] = v; }
};
struct RegWinRef {
    const RegWin &win;
    __device__ __forceinline__ float2 sample(int s) const { return win.smp[s]; }
    __device__ __forceinline__ float4 row(int r) const { return win.rc[r]; }
};

// LDS block of kWinStride float2: the entries s with s mod stride == phase (the lanes of a pixel split the writes)
struct LdsWinSink {
    float2 *rw;
    int phase, stride;
    __device__ __forceinline__ void sample(int s, float2 v) const {
        if ((s % stride) == phase) rw[s] = v;
    }
    __device__ __forceinline__ void row(int r, float4 v) const {
        if ((r % stride) == phase) reinterpret_cast<float4 *>(rw + 36)[r] = v;
    }
};

template <typename Reader>
__device__ __forceinline__ WinStats build_window(const Reader &rd, const MethodDev &m, float2 *rw, int write_phase,
                                                 int write_stride) {
    LdsWinSink sink{rw, write_phase, write_stride};
    return build_window_to(rd, m, sink);
}

// Reader of a window block in LDS for the source loop.
struct LdsWin {
    const float2 *__restrict__ rw;
    __device__ __forceinline__ float2 sample(int s) const { return rw[s]; }
    __device__ __forceinline__ float4 row(int r) const { return reinterpret_cast<const float4 *>(rw + 36)[r]; }
};


// ---------------------------------------------------------------------------
// Bilaterally weighted NCC of one hypothesis on one source (Sec. 3.3, Eq. 8).
// The window centre is projected in double precision and the warp is
// re-expressed relative to the integer texel under it, so the 36 sample
// positions keep ~1e-6 px precision in float at any image size.  Source
// moments are exact two-pass (mean first, then centred sums).
//   q0, qu, qv: inverse depth of the plane along the pixel ray and its
//   change per reference pixel in x and y.
// ---------------------------------------------------------------------------
// Source moments of the 36 samples, row by row (see ncc_cost); CLAMP as in issue_row.
template <int HALF, bool CLAMP, typename Win>
__device__ __forceinline__ void window_moments(const void *__restrict__ quads, const Win &win,
                                               float N0x, float N0y, float Z0, float pux, float puy, float puz,
                                               float pvx, float pvy, float pvz, int xlo, int xhi, int ylo, int yhi,
                                               int row_bytes, int base, float &m2, float &cab) {
    // every operation rounded as written (see build_window_to); the products with the unrounded row mean
    // are explicit fused multiply-adds
#pragma clang fp contract(off)
    // Source moments row by row: the 6 samples of a window row are held, their weighted mean,
    // centred square sum and cross sum with the reference formed exactly (two passes over the
    // row), and the rows merged with the parallel-variance update (Chan, Golub, LeVeque):
    //   mean' = mean + (mu_r - mean) W_r / W_<=r,
    //   M2'   = M2 + M2_r + (mu_r - mean)^2 W_<r W_r / W_<=r,
    //   C'    = C + C_r + (mu_r - mean') A_r + (mean - mean') A_<r.
    // No cancellation at any size of the offsets, and only 6 samples live at a time.
    float mu = 0.f, acum = 0.f;
    m2 = 0.f;
    cab = 0.f;
    // software pipeline: the gathers of row sv + 1 are issued before row sv's moments
    typename QuadT<HALF>::type qd[6];
    float fxs[6], fys[6];
    issue_row<HALF, CLAMP>(quads, -5.f, N0x, N0y, Z0, pux, puy, puz, pvx, pvy, pvz, xlo, xhi, ylo, yhi, row_bytes,
                           base, qd, fxs, fys);
#pragma unroll
    for (int sv = 0; sv < 6; ++sv) {
        float v6[6];
        float srow = 0.f;
#pragma unroll
        for (int su = 0; su < 6; ++su) {
            v6[su] = eval_quad<HALF>(qd[su], fxs[su], fys[su]);
            srow = fmaf(win.sample(sv * 6 + su).x, v6[su], srow);
        }
        if (sv < 5)
            issue_row<HALF, CLAMP>(quads, -3.f + 2.f * sv, N0x, N0y, Z0, pux, puy, puz, pvx, pvy, pvz, xlo, xhi, ylo,
                                   yhi, row_bytes, base, qd, fxs, fys);
        const float4 rc = win.row(sv);
        // mu_r = srow / W_r enters unrounded: d = v - mu_r, delta = mu_r - mean and mu_r - mean' in one rounding
        float m2r = 0.f, cr = 0.f;
#pragma unroll
        for (int su = 0; su < 6; ++su) {
            const float2 wa = win.sample(sv * 6 + su);
            const float d = fmaf(-srow, rc.x, v6[su]);
            m2r = fmaf(wa.x * d, d, m2r);
            cr = fmaf(wa.y, d, cr);
        }
        const float delta = fmaf(srow, rc.x, -mu);
        const float mun = fmaf(delta, rc.y, mu);
        m2 += fmaf(rc.z * delta, delta, m2r);
        cab += fmaf(fmaf(srow, rc.x, -mun), rc.w, fmaf(mu - mun, acum, cr));
        acum += rc.w;
        mu = mun;
    }
}

// An evaluation whose cost 2 is decided before any sample is taken (plane depth out of range at the pixel,
// window centre behind the source camera or outside its image, a window corner not in front of it) returns
// kShort from ncc_cost_raw; callers that count such evaluations map it to 2 with short_to_cost, which adds
// it to an LDS counter (carrying the flag in the result keeps a register free in the sample loop).
constexpr float kShort = -1.f;

__device__ __forceinline__ float short_to_cost(float c, unsigned *nshort) {
    if (c < 0.f) {
        atomicAdd(nshort, 1u);
        return 2.f;
    }
    return c;
}

// The warp of a window onto one source, relative to the texel (ix, iy) its centre is re-centred on: the
// homogeneous position of window offset (u, v) is N0 + u Pu + v Pv, texel indices are clamped to
// [xlo, xhi] x [ylo, yhi], and a texel's byte offset is base + yrel * row_bytes + xrel * entry bytes.
struct SrcWarp {
    float N0x, N0y, Z0, pux, puy, puz, pvx, pvy, pvz;
    int xlo, xhi, ylo, yhi, row_bytes, base;
    bool interior;  // every texel index is inside the layout without clamping
};

// False where the evaluation is decided before any sample is taken (cost kShort).
template <int HALF>
__device__ __forceinline__ bool src_warp(const ViewDev &vw, int x, int y, double q0, float qu, float qv,
                                         SrcWarp &w) {
    const double P0x = fma(vw.A[1], (double)y, fma(vw.A[0], (double)x, vw.A[2])) + vw.b[0] * q0;
    const double P0y = fma(vw.A[4], (double)y, fma(vw.A[3], (double)x, vw.A[5])) + vw.b[1] * q0;
    const double P0z = fma(vw.A[7], (double)y, fma(vw.A[6], (double)x, vw.A[8])) + vw.b[2] * q0;
    if (!(P0z > 0.0)) return false;
    const int W = vw.W, H = vw.H;
    // centre inside the source: 0 <= P0x / P0z <= W - 1 with P0z > 0, tested without a division
    if (!(P0x >= 0.0 && P0x <= (double)(W - 1) * P0z && P0y >= 0.0 && P0y <= (double)(H - 1) * P0z))
        return false;
    // the texel the window is re-centred on need not be the exact floor of the centre: everything below is
    // relative to it (N0 = P0 - (ix, iy) P0z in double, the bound on the sample offsets includes |N0|), so a
    // float estimate serves; it lies in [-1, W - 1] x [-1, H - 1] (the estimate is a few 1e-3 px off at most)
    const float rzf = __builtin_amdgcn_rcpf((float)P0z);
    const int ix = (int)floorf((float)P0x * rzf), iy = (int)floorf((float)P0y * rzf);
    w.N0x = (float)(P0x - (double)ix * P0z);
    w.N0y = (float)(P0y - (double)iy * P0z);
    w.Z0 = (float)P0z;
    w.puz = (float)vw.A[6] + (float)vw.b[2] * qu;
    w.pvz = (float)vw.A[7] + (float)vw.b[2] * qv;
    w.pux = (float)vw.A[0] + (float)vw.b[0] * qu - (float)ix * w.puz;
    w.puy = (float)vw.A[3] + (float)vw.b[1] * qu - (float)iy * w.puz;
    w.pvx = (float)vw.A[1] + (float)vw.b[0] * qv - (float)ix * w.pvz;
    w.pvy = (float)vw.A[4] + (float)vw.b[1] * qv - (float)iy * w.pvz;
    // every sample must see the plane in front of the source camera: the depth is affine in the
    // window offsets, so the four corners decide
    const float zc0 = w.Z0 - 5.f * w.puz - 5.f * w.pvz, zc1 = w.Z0 + 5.f * w.puz - 5.f * w.pvz;
    const float zc2 = w.Z0 - 5.f * w.puz + 5.f * w.pvz, zc3 = w.Z0 + 5.f * w.puz + 5.f * w.pvz;
    if (!(fminf(fminf(zc0, zc1), fminf(zc2, zc3)) > 1e-20f)) return false;

    // texel indices relative to (ix, iy), clamped to [-1, W-1] x [-1, H-1] in absolute terms;
    // byte offset = base + yrel * row_bytes + xrel * entry_bytes (non-negative after clamping)
    constexpr int kEntry = HALF ? 4 : 8;
    w.row_bytes = (W + 2 + 2 * kQuadPad) * kEntry;
    w.xlo = -1 - ix;
    w.xhi = W - 1 - ix;
    w.ylo = -1 - iy;
    w.yhi = H - 1 - iy;
    w.base = ((iy + 1 + kQuadPad) * (W + 2 + 2 * kQuadPad) + (ix + 1 + kQuadPad)) * kEntry;
    // Clamp-free fast path: the samples lie in the convex image of the window square (the depth is
    // positive at its corners, so the warp has no pole inside), hence |dx| <= (|N0x| + 5 |pux| + 5 |pvx|)
    // / min corner depth, likewise dy.  When that bound (widened by 1 % + 0.01 px, far above the float
    // rounding of the samples once the min depth exceeds 1e-3 of the centre's) keeps every texel index
    // inside the layout (the clamp range widened by its border), the clamps are skipped: inside the clamp
    // range they change nothing, and the border holds the clamped footprint: the same values, the same result.
    const float zmin = fminf(fminf(zc0, zc1), fminf(zc2, zc3));
    const float rzm = __builtin_amdgcn_rcpf(zmin);
    const float bx = fmaf(fmaf(5.f, fabsf(w.pux) + fabsf(w.pvx), fabsf(w.N0x)) * rzm, 1.01f, 0.01f);
    const float by = fmaf(fmaf(5.f, fabsf(w.puy) + fabsf(w.pvy), fabsf(w.N0y)) * rzm, 1.01f, 0.01f);
    // (the border of the layout extends the clamp-free range by kQuadPad texels on every side)
    w.interior = zmin > 1e-3f * w.Z0 && bx <= (float)(ix + 1 + kQuadPad) && bx < (float)(W - ix + kQuadPad) &&
                 by <= (float)(iy + 1 + kQuadPad) && by < (float)(H - iy + kQuadPad);
    return true;
}

// The cost from the source moments: 1 - NCC, clamped to [0, 2]; 2 for a textureless window on either side.
__device__ __forceinline__ float cost_from_moments(const WinStats &ws, float m2, float cab) {
    const float var_b = m2 * ws.invW;
    const float cov = cab * ws.invW;
    if (ws.var_a < 1e-5f || var_b < 1e-5f) return 2.f;
    const float mm = 1.f - cov * rsqrtf(ws.var_a * var_b);
    return fminf(fmaxf(mm, 0.f), 2.f);
}

template <int HALF, bool SPLIT, typename Win>
__device__ __forceinline__ float ncc_cost_win(const ViewDev &vw, const Win &rw, const WinStats &ws, int x, int y,
                                              double q0, float qu, float qv) {
    SrcWarp w;
    if (!src_warp<HALF>(vw, x, y, q0, qu, qv, w)) return kShort;
    // SPLIT = false: every lane takes the clamped path, which gives interior lanes the same result.  A wave
    // whose lanes disagree runs both paths in turn, so where the hypotheses are random (steep planes, windows
    // at the image edges: the two mix in nearly every wave) the clamped path alone is the cheaper one.
    float m2, cab;
    if (SPLIT && w.interior)
        window_moments<HALF, false>(vw.quads, rw, w.N0x, w.N0y, w.Z0, w.pux, w.puy, w.puz, w.pvx, w.pvy, w.pvz,
                                    w.xlo, w.xhi, w.ylo, w.yhi, w.row_bytes, w.base, m2, cab);
    else
        window_moments<HALF, true>(vw.quads, rw, w.N0x, w.N0y, w.Z0, w.pux, w.puy, w.puz, w.pvx, w.pvy, w.pvz,
                                   w.xlo, w.xhi, w.ylo, w.yhi, w.row_bytes, w.base, m2, cab);
    return cost_from_moments(ws, m2, cab);
}

template <int HALF, bool SPLIT = true>
__device__ __forceinline__ float ncc_cost_raw(const ViewDev &vw, const float2 *__restrict__ rw, const WinStats &ws,
                                              int x, int y, double q0, float qu, float qv) {
    return ncc_cost_win<HALF, SPLIT>(vw, LdsWin{rw}, ws, x, y, q0, qu, qv);
}

// The cost with short evaluations not counted.
template <int HALF>
__device__ __forceinline__ float ncc_cost(const ViewDev &vw, const float2 *__restrict__ rw, const WinStats &ws, int x,
                                          int y, double q0, float qu, float qv) {
    const float c = ncc_cost_raw<HALF>(vw, rw, ws, x, y, q0, qu, qv);
    return c < 0.f ? 2.f : c;
}

// ---------------------------------------------------------------------------
// One evaluation on a pair of lanes (lanes 2i, 2i + 1 of a wave, the same
// pixel and hypothesis): lane h takes the window columns h, h + 2, h + 4 of
// every row, so that the two loads a pair issues together fall on
// neighbouring texels of one source row (where hypotheses are random, a wave
// whose 64 lanes each gather their own window touches 64 cache lines per
// load instruction).  The warp setup and the row merge are computed by both
// lanes alike (the same values, bit for bit, so the pair never diverges); the
// row sums are exchanged within the pair, and each lane's part of the second
// moments is summed at the end.
// ---------------------------------------------------------------------------
// the value held by the other lane of the pair
__device__ __forceinline__ float pair_other(float v) {
    // quad permutation (1, 0, 3, 2)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// The half of a pixel's window block that one lane of the pair holds: the entries of its 18 samples (sample
// s = 6 row + column, the lane's are those with s mod 2 = h, at s / 2) and the 6 row constants, with the two
// merge terms (W_<r W_r / W_<=r, A_r) zeroed in lane 1 so that each row's cross terms enter once.
struct PairWin {
    float2 smp[18];
    float4 rc[6];
};
struct PairWinSink {
    PairWin *win;
    bool odd;
    __device__ __forceinline__ void sample(int s, float2 v) const {
        if ((s & 1) == 0 || odd) win->smp[s >> 1] = v;
    }
    __device__ __forceinline__ void row(int r, float4 v) const {
        win->rc[r] = odd ? make_float4(v.x, v.y, 0.f, 0.f) : v;
    }
};

// the gathers of the lane's 3 samples of window row vf (offsets uf[k] = -5 + 2 h + 4 k), always clamped
template <int HALF>
__device__ __forceinline__ void issue_cols(const void *quads, float vf, const float (&uf)[3], const SrcWarp &w,
                                           typename QuadT<HALF>::type (&qd)[3], float (&fxs)[3], float (&fys)[3]) {
    constexpr int kEntry = HALF ? 4 : 8;
    const float rx = fmaf(vf, w.pvx, w.N0x), ry = fmaf(vf, w.pvy, w.N0y), rzz = fmaf(vf, w.pvz, w.Z0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float nx = fmaf(uf[k], w.pux, rx), ny = fmaf(uf[k], w.puy, ry), nz = fmaf(uf[k], w.puz, rzz);
        const float r = __builtin_amdgcn_rcpf(nz);
        const float dx = nx * r, dy = ny * r;
        const int xr = med3i(cvt_floor(dx), w.xlo, w.xhi);
        const int yr = med3i(cvt_floor(dy), w.ylo, w.yhi);
        fxs[k] = __builtin_amdgcn_fractf(dx);
        fys[k] = __builtin_amdgcn_fractf(dy);
        const uint32_t off = (uint32_t)__mul24(yr, w.row_bytes) + (uint32_t)w.base + (uint32_t)xr * kEntry;
        qd[k] = load_quad<HALF>(quads, off);
    }
}

// Source moments of the window on the pair, row by row as in window_moments: the row mean needs the row's
// weighted sum over both lanes; the centred sums over the lane's 3 samples and the merge terms (zero in
// lane 1) accumulate per lane and are added over the pair at the end.
template <int HALF>
__device__ __forceinline__ void pair_moments(const void *__restrict__ quads, const PairWin &win,
                                             const float (&uf)[3], const SrcWarp &w, float &m2, float &cab) {
#pragma clang fp contract(off)
    float mu = 0.f, acum = 0.f;
    m2 = 0.f;
    cab = 0.f;
    typename QuadT<HALF>::type qd[3];
    float fxs[3], fys[3];
    issue_cols<HALF>(quads, -5.f, uf, w, qd, fxs, fys);
#pragma unroll
    for (int sv = 0; sv < 6; ++sv) {
        float v3[3];
        float sp = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v3[k] = eval_quad<HALF>(qd[k], fxs[k], fys[k]);
            sp = fmaf(win.smp[sv * 3 + k].x, v3[k], sp);
        }
        if (sv < 5) issue_cols<HALF>(quads, -3.f + 2.f * sv, uf, w, qd, fxs, fys);
        // the same sum in both lanes (addition commutes bit for bit)
        const float srow = sp + pair_other(sp);
        const float4 rc = win.rc[sv];
        float m2r = 0.f, cr = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float2 wa = win.smp[sv * 3 + k];
            const float d = fmaf(-srow, rc.x, v3[k]);
            m2r = fmaf(wa.x * d, d, m2r);
            cr = fmaf(wa.y, d, cr);
        }
        const float delta = fmaf(srow, rc.x, -mu);
        const float mun = fmaf(delta, rc.y, mu);
        m2 += fmaf(rc.z * delta, delta, m2r);
        cab += fmaf(fmaf(srow, rc.x, -mun), rc.w, fmaf(mu - mun, acum, cr));
        acum += rc.w;
        mu = mun;
    }
    m2 += pair_other(m2);
    cab += pair_other(cab);
}

template <int HALF>
__device__ __forceinline__ float ncc_cost_pair(const ViewDev &vw, const PairWin &win, const WinStats &ws, int x,
                                               int y, double q0, float qu, float qv, const float (&uf)[3]) {
    SrcWarp w;
    if (!src_warp<HALF>(vw, x, y, q0, qu, qv, w)) return kShort;
    float m2, cab;
    pair_moments<HALF>(vw.quads, win, uf, w, m2, cab);
    return cost_from_moments(ws, m2, cab);
}

// inverse-depth terms of a plane at reference pixel (x, y): q = -(n . K^-1 (x, y, 1)) / d
struct PlaneQ {
    double q0;
    float qu, qv;
    bool ok;  // depth at the pixel inside [d_min, d_max]
};

__device__ __forceinline__ PlaneQ plane_q(const RefDev &ref, const MethodDev &m, float4 pl, int x, int y) {
    const double rx = fma(ref.kinv_a, (double)x, fma(ref.kinv_b, (double)y, ref.kinv_c));
    const double ry = fma(ref.kinv_e, (double)y, ref.kinv_f);
    const double nr = (double)pl.x * rx + (double)pl.y * ry + (double)pl.z;
    const double d = (double)pl.w;
    PlaneQ q;
    const double inv_d = -1.0 / d;  // the one division: q0 = -nr / d is the inverse depth at the pixel
    q.q0 = nr * inv_d;
    // range test on the inverse depth, with a relative tolerance of 1e-5 on the depth (refinement clamps
    // depths to the ends of the range, and the plane rebuilt from a clamped depth must not fail on its last
    // bit); q_lo > 0, so a depth behind the camera fails too
    q.ok = q.q0 >= m.q_lo && q.q0 <= m.q_hi;
    const float invd = (float)inv_d;
    q.qu = (float)(pl.x * ref.kinv_a) * invd;
    q.qv = (float)(pl.x * ref.kinv_b + pl.y * ref.kinv_e) * invd;
    // every window sample's ray must meet the plane in front of the camera: the inverse depth is
    // affine in the window offsets, so the four corners decide
    const float qc = (float)q.q0, hu = 5.f * q.qu, hv = 5.f * q.qv;
    q.ok = q.ok && fminf(fminf(qc - hu - hv, qc + hu - hv), fminf(qc - hu + hv, qc + hu + hv)) > 0.f;
    return q;
}

// viewing ray K_ref^-1 (x, y, 1) of a reference pixel (its z component is 1)
__device__ __forceinline__ float2 ref_ray(const RefDev &ref, int x, int y) {
    return make_float2((float)fma(ref.kinv_a, (double)x, fma(ref.kinv_b, (double)y, ref.kinv_c)),
                       (float)fma(ref.kinv_e, (double)y, ref.kinv_f));
}

// plane through the point at `depth` on the ray r with normal n turned to face the camera
__device__ __forceinline__ float4 plane_from(float2 r, float depth, float nx, float ny, float nz) {
    float nr = nx * r.x + ny * r.y + nz;
    if (nr > 0.f) {
        nx = -nx; ny = -ny; nz = -nz; nr = -nr;
    }
    return make_float4(nx, ny, nz, -depth * nr);
}

// uniform direction on the sphere: z = 1 - 2 u1, azimuth 2 pi u2
__device__ __forceinline__ void normal_from_uniforms(float u1, float u2, float &nx, float &ny, float &nz) {
    const float z = 1.f - 2.f * u1;
    const float s = sqrtf(fmaxf(0.f, 1.f - z * z));
    float sn, cs;
    sincospif(2.f * u2, &sn, &cs);
    nx = s * cs; ny = s * sn; nz = z;
}

__device__ __forceinline__ float plane_depth(float2 r, float4 pl) {
    return -pl.w / (pl.x * r.x + pl.y * r.y + pl.z);
}

// ---------------------------------------------------------------------------
// Tile mapping.  Workgroups are spread round-robin over the 8 XCDs; logical
// tiles are renumbered so that each XCD walks a contiguous band of rows and
// keeps its sources' footprint in its own L2.
// ---------------------------------------------------------------------------
// order 0: XCD bands (block b runs on XCD b mod 8 and takes the (b / 8)-th tile of
// that XCD's band); order 1: hardware order (block b takes tile b).
__device__ __forceinline__ int tile_of_block(int n_tiles, int order) {
    const int b = blockIdx.x;
    if (order == 1) return b < n_tiles ? b : -1;
    const int per = (n_tiles + 7) >> 3;
    const int L = (b & 7) * per + (b >> 3);
    return L < n_tiles ? L : -1;
}

// LDS carve-up of the pass / init kernels
struct PassLds {
    float *tile;     // WAVES + 10 rows x (2 * kTilePix + 10) cols of reference intensities
    float2 *rw;      // [wave][group][kWinStride] window blocks
    float4 *pl;      // [256] hypothesis of each lane
    float *ms;       // [wave][n_src][64] costs, reused for refinement results
    float *mf;       // [256] aggregated cost / scratch
    float *psi;      // [wave][group][32] importance, < 0 outside S_t
    int *valid;      // [256]
    unsigned char *act;  // [wave][group][32] active views for refinement
    float4 *cand;    // [wave][group][6] refinement candidates
    float *wgt;      // [wave][group][32] view weights of each pixel
    unsigned *nshort;  // [wave] evaluations of the wave that took no samples (touched by that wave only)
    int *gnw;          // [wave][8] refinement: active views of each pixel of the wave (0: no pixel)
    float2 *gws;       // [wave][8] ... and its window statistics (1 / sum w, weighted reference variance)
};

constexpr int kTileW = 2 * kTilePix + 10;

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// LDS of a workgroup of `waves` waves (one image row of the tile per wave); rb row blocks of the 9 lanes of
// a pixel (1; 3 for the 21 rows of the standard symmetric pattern) for the hypotheses, their validity, the
// cost matrix and the aggregated costs, block b at offset b * waves * 64 entries
__host__ __device__ inline size_t lds_layout(int n_src, int waves, size_t off[13], int rb = 1) {
    size_t o = 0;
    off[0] = o; o = align16(o + sizeof(float) * (waves + 10) * kTileW);
    off[1] = o; o = align16(o + sizeof(float2) * waves * kGroups * kWinStride);
    off[2] = o; o = align16(o + sizeof(float4) * rb * waves * 64);
    off[3] = o; o = align16(o + sizeof(float) * rb * waves * (n_src > 7 ? n_src : 7) * 64);
    off[4] = o; o = align16(o + sizeof(float) * rb * waves * 64);
    off[5] = o; o = align16(o + sizeof(float) * waves * kGroups * kMaxSrc);
    off[6] = o; o = align16(o + sizeof(int) * rb * waves * 64);
    off[7] = o; o = align16(o + waves * kGroups * kMaxSrc);
    off[8] = o; o = align16(o + sizeof(float4) * waves * kGroups * 6);
    off[9] = o; o = align16(o + sizeof(float) * waves * kGroups * kMaxSrc);
    off[10] = o; o = align16(o + sizeof(unsigned) * waves);
    off[11] = o; o = align16(o + sizeof(int) * waves * 8);
    off[12] = o; o = align16(o + sizeof(float2) * waves * 8);
    return o;
}

size_t pass_lds_bytes(int n_src, int waves, int rb) {
    size_t off[13];
    return lds_layout(n_src, waves, off, rb);
}

__device__ __forceinline__ PassLds carve(unsigned char *smem, int n_src, int waves, int rb = 1) {
    size_t off[13];
    lds_layout(n_src, waves, off, rb);
    PassLds L;
    L.tile = reinterpret_cast<float *>(smem + off[0]);
    L.rw = reinterpret_cast<float2 *>(smem + off[1]);
    L.pl = reinterpret_cast<float4 *>(smem + off[2]);
    L.ms = reinterpret_cast<float *>(smem + off[3]);
    L.mf = reinterpret_cast<float *>(smem + off[4]);
    L.psi = reinterpret_cast<float *>(smem + off[5]);
    L.valid = reinterpret_cast<int *>(smem + off[6]);
    L.act = smem + off[7];
    L.cand = reinterpret_cast<float4 *>(smem + off[8]);
    L.wgt = reinterpret_cast<float *>(smem + off[9]);
    L.nshort = reinterpret_cast<unsigned *>(smem + off[10]);
    L.gnw = reinterpret_cast<int *>(smem + off[11]);
    L.gws = reinterpret_cast<float2 *>(smem + off[12]);
    return L;
}

// reference tile of a workgroup: rows y0-5 .. y0+WAVES+4, cols x0-5 .. x0+2*kTilePix+4, clamped
template <int WAVES>
__device__ __forceinline__ void stage_tile(const RefDev &ref, float *tile, int y0, int x0, int tid) {
    for (int i = tid; i < (WAVES + 10) * kTileW; i += 64 * WAVES) {
        const int ty = i / kTileW, tx = i - ty * kTileW;
        const int gy = min(max(y0 - 5 + ty, 0), ref.H - 1);
        const int gx = min(max(x0 - 5 + tx, 0), ref.W - 1);
        tile[i] = glob(ref.img)[(size_t)gy * ref.W + gx];
    }
}

struct TileReader {
    const float *tile;
    int cy, cx;  // pixel position inside the tile
    const RefDev *ref;
    int x, y;
    __device__ __forceinline__ float operator()(int du, int dv) const {
        // clamp to the image exactly like the global reader: positions are clamped in image space
        const int gx = min(max(x + du, 0), ref->W - 1), gy = min(max(y + dv, 0), ref->H - 1);
        return tile[(cy + (gy - y)) * kTileW + (cx + (gx - x))];
    }
};

struct GlobalReader {
    const RefDev *ref;
    int x, y;
    __device__ __forceinline__ float operator()(int du, int dv) const {
        const int gx = min(max(x + du, 0), ref->W - 1), gy = min(max(y + dv, 0), ref->H - 1);
        return ref->img[(size_t)gy * ref->W + gx];
    }
};

__device__ __forceinline__ void count_evals(unsigned long long *counters, int kind, unsigned long long n) {
    // one atomic per wave, spread over slots
    const int lane = threadIdx.x & 63;
    unsigned long long tot = n;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_down(tot, off, 64);
    if (lane == 0 && tot)
        atomicAdd(&counters[kind * kCounterSlots + ((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kCounterSlots)],
                  tot);
}

// ---------------------------------------------------------------------------
// Plane of pixel (x, y) from the prediction of its s x s cell (s = a.prop_s: 4
// for the learned proposal, 1 for per-pixel hypotheses): through the point at
// the predicted depth on the ray of the cell's sample pixel (s j + s / 2,
// s i + s / 2, clamped to the image), with the predicted normal turned to
// face the pixel's ray.  False (keep the random
// plane) when the confidence is below conf_min, the normal is zero or not
// finite, or the plane's depth along the pixel's ray leaves [d_min, d_max].
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool proposal_plane(const PassArgs &a, float2 r, int x, int y, float4 &pl) {
    // explicit fused multiply-adds: the two initialisation kernels inline this function, and the
    // result must not depend on how the compiler contracts it at each call site
    const int cs = a.prop_s;
    const int i = y / cs, j = x / cs;
    const float *pp = a.prop + ((size_t)i * a.prop_w + j) * 5;
    const float depth = pp[0], conf = pp[4];
    float nx = pp[1], ny = pp[2], nz = pp[3];
    const float nn = __builtin_sqrtf(fmaf(nx, nx, fmaf(ny, ny, __fmul_rn(nz, nz))));
    if (!(conf >= a.conf_min) || !(nn > 0.f) || !__builtin_isfinite(nn) || !__builtin_isfinite(depth)) return false;
    nx /= nn;
    ny /= nn;
    nz /= nn;
    const float2 rc = ref_ray(a.ref, min(cs * j + cs / 2, a.ref.W - 1), min(cs * i + cs / 2, a.ref.H - 1));
    float dp = __fmul_rn(-depth, fmaf(nx, rc.x, fmaf(ny, rc.y, nz)));
    float nr = fmaf(nx, r.x, fmaf(ny, r.y, nz));
    if (nr > 0.f) {
        nx = -nx;
        ny = -ny;
        nz = -nz;
        dp = -dp;
        nr = -nr;
    }
    if (!(nr < 0.f)) return false;
    const float d = -dp / nr;
    if (!(d >= a.m.d_min && d <= a.m.d_max)) return false;
    pl = make_float4(nx, ny, nz, dp);
    return true;
}

// ---------------------------------------------------------------------------
// Initialisation of one colour with one pixel per pair of lanes (see
// ncc_cost_pair): each lane of the pair builds the pixel's window block and
// keeps its half in registers, and the wave walks the sources together (the
// view's warp constants in scalar registers, as in the pass).  kInitBlock
// pixels of the colour per workgroup of 2 kInitBlock lanes, in row-major
// order, workgroups in XCD bands; the costs go to LDS, one row per source,
// and the pair's even lane takes the mean of the k lowest.  The batched
// initialisation runs the same body, so a job's initial state is the same
// bits either way.
// ---------------------------------------------------------------------------
// Block blk (of init_blocks) of the colour: cst is [n_src][kInitBlock] floats of LDS, nshort an LDS counter.
template <int HALF>
__device__ __forceinline__ void init_pair_body(const PassArgs &a, long long blk, float *cst, unsigned *nshort_p) {
    unsigned &nshort = *nshort_p;
    const int N = a.n_src;
    const int t = threadIdx.x, pi = t >> 1;
    const bool odd = (t & 1) != 0;
    const int per_row = (a.ref.W + 1) / 2;  // slots per row; x beyond the image is skipped
    const long long pc = blk * kInitBlock + pi;
    const int y = (int)(pc / per_row);
    const int x = 2 * (int)(pc - (long long)y * per_row) + ((y + a.colour) & 1);
    const bool pix_ok = y < a.ref.H && x < a.ref.W;
    if (t == 0) nshort = 0u;
    PairWin win;
    WinStats ws = {1.f, 0.f};
    float4 pl = make_float4(0.f, 0.f, -1.f, 1.f);
    bool fell_back = false;
    PlaneQ q;
    q.ok = false;
    if (pix_ok) {
        GlobalReader rd{&a.ref, x, y};
        PairWinSink sink{&win, odd};
        ws = build_window_to(rd, a.m, sink);
        const float2 r = ref_ray(a.ref, x, y);
        if (!(a.prop && proposal_plane(a, r, x, y, pl))) {
            fell_back = a.prop != nullptr;
            float u[4], nx, ny, nz;
            philox((uint64_t)y * a.ref.W + x, 0, 0, a.m.seed, u);
            const float depth = a.m.d_min + u[0] * (a.m.d_max - a.m.d_min);
            normal_from_uniforms(u[1], u[2], nx, ny, nz);
            pl = plane_from(r, depth, nx, ny, nz);
        }
        q = plane_q(a.ref, a.m, pl, x, y);
        // the plane is final: store it now, so that it is not held through the source loop
        if (!odd) store_plane(a.st.planes, (size_t)y * a.ref.W + x, pl);
    }
    const float u0 = odd ? -3.f : -5.f;
    const float uf[3] = {u0, u0 + 4.f, u0 + 8.f};
    __syncthreads();
    for (int j = 0; j < N; ++j) {
        if (pix_ok) {
            const float c = q.ok ? ncc_cost_pair<HALF>(a.views[j], win, ws, x, y, q.q0, q.qu, q.qv, uf) : kShort;
            if (!odd) cst[j * kInitBlock + pi] = short_to_cost(c, &nshort);
        }
    }
    const bool counts = pix_ok && !odd;
    count_evals(a.counters, 0, counts ? (unsigned long long)N : 0ull);
    if (a.prop) count_evals(a.counters, 3, counts && fell_back ? 1ull : 0ull);
    if (counts) {
        // mean of the k lowest costs, in ascending order (each lane reads only the costs it wrote)
        const int kk = a.m.k < N ? a.m.k : N;
        uint32_t taken = 0;
        float sum = 0.f;
        for (int r = 0; r < kk; ++r) {
            int best = -1;
            float bc = 0.f;
            for (int v = 0; v < N; ++v) {
                if ((taken >> v) & 1u) continue;
                const float c = cst[v * kInitBlock + pi];
                if (best < 0 || c < bc) {
                    best = v;
                    bc = c;
                }
            }
            taken |= 1u << best;
            sum += bc;
        }
        const size_t p = (size_t)y * a.ref.W + x;
        glob(a.st.cost)[p] = sum / (float)kk;
        glob(a.st.S)[p] = 0u;
        glob(a.st.v)[p] = -1;
    }
    __syncthreads();
    count_evals(a.counters, 5, t == 0 ? (unsigned long long)nshort : 0ull);
}

template <int HALF>
__global__ __launch_bounds__(2 * kInitBlock) __attribute__((amdgpu_waves_per_eu(AMH_INIT_WAVES_PER_EU))) void
init_pair_kernel(PassArgs a) {
    extern __shared__ __align__(16) float cst[];  // [n_src][kInitBlock]
    __shared__ unsigned nshort;
    // XCD bands: block b runs on XCD b mod 8 and takes the (b / 8)-th block of that XCD's band
    const long long n_blocks = init_blocks(a.ref.W, a.ref.H);
    const long long per_xcd = (n_blocks + 7) >> 3;
    const long long blk = (long long)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (blk >= n_blocks) return;  // the whole workgroup leaves before any barrier
    init_pair_body<HALF>(a, blk, cst, &nshort);
}

// ---------------------------------------------------------------------------
// One checkerboard half-pass (Sec. 3.1 - 3.3).
// ---------------------------------------------------------------------------
// A weighted refinement cost w * m as stored: a short evaluation is stored as w * kShort = -w, its cost is 2 w.
__device__ __forceinline__ float weighted_cost(float r) { return r < 0.f ? -2.f * r : r; }

// Mean of the kk lowest of n values at stride `stride` (heuristic view selection of the ablation); the
// values are costs, or weighted costs as stored by refinement.
__device__ __forceinline__ float mean_k_lowest(const float *c, int stride, int n, int kk) {
    uint32_t taken = 0;
    float sum = 0.f;
    for (int r = 0; r < kk; ++r) {
        int bj = -1;
        float bv = 0.f;
        for (int j = 0; j < n; ++j) {
            if ((taken >> j) & 1u) continue;
            const float v = weighted_cost(c[j * stride]);
            if (bj < 0 || v < bv) { bj = j; bv = v; }
        }
        taken |= 1u << bj;
        sum += bv;
    }
    return sum / (float)kk;
}

// Standard symmetric checkerboard pattern (Fig. 2(b), ablation): neighbour R (0..19) in the order of a
// row-major scan of the 11 x 11 square around the pixel over the other-colour pixels within L1 distance 3 and
// the four axial ones at distance 5.
__device__ __forceinline__ void std_offset(int R, int &dx, int &dy) {
    int n = 0;
    dx = 0;
    dy = 0;
    for (int oy = -5; oy <= 5; ++oy)
        for (int ox = -5; ox <= 5; ++ox) {
            const int l1 = abs(ox) + abs(oy);
            if (!(l1 & 1) || !(l1 <= 3 || (l1 == 5 && (ox == 0 || oy == 0)))) continue;
            if (n == R) {
                dx = ox;
                dy = oy;
            }
            ++n;
        }
}
constexpr int kStdRows = 20;  // propagated rows of the standard symmetric pattern; row 20 is the own plane

// ABL: the ablation build of the pass, with the two switches of Sec. 4 read at run
// time: m.sym_prop (symmetric checkerboard propagation: 1, region r holds the one
// neighbour at distance 1 (r < 4) or 5 (r >= 4) up/down/left/right, the fast
// pattern of Fig. 2(c); 2, the 20 neighbours of the standard pattern of
// Fig. 2(b), in three blocks of 9 rows per pixel: row R = 9 b + lane row, the
// own plane at R = 20, and the view selection's counts n1, n2 compared as the
// same fractions of 20 rows as of 8) and m.heuristic (each hypothesis, and each refinement
// candidate, costs the mean of its own k lowest per-view costs; no selection memory).
// tid: threadIdx.x (the persistent launch passes it through an opaque copy, so that nothing derived from
// it is kept live across its tiles)
template <int HALF, int WAVES, bool ABL = false>
__device__ __forceinline__ void pass_body(const PassArgs &a, int L, unsigned char *smem, int tid) {
    // row blocks: 3 in the standard symmetric pattern (ablation build only), else 1
    const bool stdp = ABL && a.m.sym_prop == 2;
    const int RB = stdp ? 3 : 1;
    PassLds S = carve(smem, a.n_src, WAVES, RB);
    constexpr int WL = 64 * WAVES;  // entries per row block of pl, valid, mf
    const int wave = tid >> 6, lane = tid & 63;
    const int grp = lane / kRows, row = lane - grp * kRows;
    const int g = grp < kGroups ? grp : 0;
    const int ty = L / a.tiles_x, tx = L - ty * a.tiles_x;
    const int y0 = ty * WAVES, x0 = tx * 2 * kTilePix;
    const int y = y0 + wave;
    const int x = 2 * (tx * kTilePix + grp) + ((y + a.colour) & 1);
    const int W = a.ref.W, H = a.ref.H;
    const bool pix_ok = grp < kGroups && y < H && x < W;
    const size_t p = pix_ok ? (size_t)y * W + x : 0;
    const int N = a.n_src;
    const MethodDev &m = a.m;

    stage_tile<WAVES>(a.ref, S.tile, y0, x0, tid);

    // (1) asymmetric propagation: lane r < 8 takes the lowest-cost candidate of region r
    float4 pl = make_float4(0.f, 0.f, -1.f, 1.f);
    bool valid = false;
    if (stdp) {
        for (int b = 0; b < 3; ++b) {
            const int R = 9 * b + row;
            float4 plb = make_float4(0.f, 0.f, -1.f, 1.f);
            bool vb = false;
            if (pix_ok && R < kStdRows) {
                int dx, dy;
                std_offset(R, dx, dy);
                const int nx = x + dx, ny = y + dy;
                if (nx >= 0 && nx < W && ny >= 0 && ny < H) {
                    vb = true;
                    plb = load_plane(a.st.planes, (size_t)ny * W + nx);
                }
            } else if (pix_ok && R == kStdRows) {
                vb = m.include_self != 0;
                plb = load_plane(a.st.planes, p);
            }
            S.pl[b * WL + tid] = plb;
            S.valid[b * WL + tid] = vb ? 1 : 0;
        }
    } else if (pix_ok) {
        if (ABL && m.sym_prop && row < 8) {
            const int u = row < 4 ? 1 : 5, dir = row & 3;
            const int nx = x + (dir == 2 ? -u : (dir == 3 ? u : 0));
            const int ny = y + (dir == 0 ? -u : (dir == 1 ? u : 0));
            if (nx >= 0 && nx < W && ny >= 0 && ny < H) {
                valid = true;
                pl = load_plane(a.st.planes, (size_t)ny * W + nx);
            }
        } else if (row < 8) {
            // the region's stored costs are loaded together (all in flight at once), then taken in table order
            const int ne = region_size(row);
            float cr[11];
            bool in[11];
#pragma unroll
            for (int e = 0; e < 11; ++e) {
                int dx, dy;
                region_offset(row, e, dx, dy);
                const int nx = x + dx, ny = y + dy;
                in[e] = e < ne && nx >= 0 && nx < W && ny >= 0 && ny < H;
                cr[e] = in[e] ? glob(a.st.cost)[(size_t)ny * W + nx] : 0.f;
            }
            int be = -1;
            float bc = 0.f;
#pragma unroll
            for (int e = 0; e < 11; ++e)
                if (in[e] && (be < 0 || cr[e] < bc)) {
                    be = e;
                    bc = cr[e];
                }
            if (be >= 0) {
                int dx, dy;
                region_offset(row, be, dx, dy);
                valid = true;
                pl = load_plane(a.st.planes, (size_t)(y + dy) * W + (x + dx));
            }
        } else {
            valid = m.include_self != 0;
            pl = load_plane(a.st.planes, p);
        }
    }
    if (!stdp) {
        S.pl[tid] = pl;
        S.valid[tid] = valid ? 1 : 0;
    }
    if (lane == 0) S.nshort[wave] = 0u;
    __syncthreads();

    // (2) reference window, split over the 9 lanes of the pixel
    float2 *rw = S.rw + (wave * kGroups + g) * kWinStride;
    WinStats ws = {1.f, 0.f};
    if (pix_ok) {
        TileReader rd{S.tile, 5 + wave, 5 + (x - x0), &a.ref, x, y};
        ws = build_window(rd, m, rw, row, kRows);
    }
    __syncthreads();

    // (3) cost matrix (Eq. 1) plus the own row: one column per view (row block b at mcol + b * WAVES * N * 64)
    float *mcol = S.ms + wave * N * 64;
    int n_prop = 0;
    for (int b = 0; b < RB; ++b) {
        float *mc = mcol + b * WAVES * N * 64;
        const float4 plb = stdp ? S.pl[b * WL + tid] : pl;
        const bool vb = stdp ? S.valid[b * WL + tid] != 0 : valid;
        const PlaneQ q = plane_q(a.ref, m, plb, x, y);
        for (int j = 0; j < N; ++j) {
            float c = 2.f;
            if (vb) {
                c = q.ok ? ncc_cost_raw<HALF>(a.views[j], rw, ws, x, y, q.q0, q.qu, q.qv) : kShort;
                ++n_prop;
            }
            mc[j * 64 + lane] = c;
        }
        // short evaluations were stored as kShort: counted and set to 2 from LDS after the loop, so that
        // the loop itself carries no counter
        if (vb) {
            unsigned ns = 0;
            for (int j = 0; j < N; ++j) {
                if (mc[j * 64 + lane] < 0.f) {
                    ++ns;
                    mc[j * 64 + lane] = 2.f;
                }
            }
            if (ns) atomicAdd(&S.nshort[wave], ns);
        }
    }
    __syncthreads();

    // (4) view inference, part 1 (Sec. 3.2): lane r judges views r, r+9, ...
    //     good view: more than n1 costs below tau and fewer than n2 above tau_up;
    //     importance: mean confidence exp(-m^2 / (2 beta^2)) over the valid rows
    float *psi = S.psi + (wave * kGroups + g) * kMaxSrc;
    const bool heur = ABL && m.heuristic;  // uniform over the launch
    int nv = 0;
    if (stdp) {
        // 20 propagated rows: row i in block i / 9, lane row i % 9; counts against n R / 8
        for (int i = 0; i < kStdRows; ++i) nv += S.valid[(i / 9) * WL + wave * 64 + g * kRows + i % 9];
        const float n1s = (float)m.n1 * (kStdRows / 8.f), n2s = (float)m.n2 * (kStdRows / 8.f);
        if (pix_ok && !heur) {
            for (int j = row; j < N; j += kRows) {
                int lt = 0, gt = 0;
                float sc = 0.f;
                for (int i = 0; i < kStdRows; ++i) {
                    const int b = i / 9, r = i % 9;
                    if (!S.valid[b * WL + wave * 64 + g * kRows + r]) continue;
                    const float c = mcol[b * WAVES * N * 64 + j * 64 + g * kRows + r];
                    lt += c < m.tau;
                    gt += c > m.tau_up;
                    sc += __expf(-c * c * m.inv_2b2);
                }
                psi[j] = (nv > 0 && (float)lt > n1s && (float)gt < n2s) ? sc / (float)nv : -1.f;
            }
        }
    } else {
        // valid propagated rows of the pixel: one ballot
        nv = __popcll((__ballot(valid && row < 8) >> (kRows * grp)) & 0xFFull);
        if (pix_ok && !heur) {
            for (int j = row; j < N; j += kRows) {
                int lt = 0, gt = 0;
                float sc = 0.f;
                for (int i = 0; i < 8; ++i) {
                    if (!S.valid[wave * 64 + g * kRows + i]) continue;
                    const float c = mcol[j * 64 + g * kRows + i];
                    lt += c < m.tau;
                    gt += c > m.tau_up;
                    sc += __expf(-c * c * m.inv_2b2);
                }
                psi[j] = (nv > 0 && lt > m.n1 && gt < m.n2) ? sc / (float)nv : -1.f;
            }
        }
    }
    __syncthreads();

    // (5) view inference, part 2 (Eq. 4-6).  Lane r of the pixel holds views r, r+9, r+18, r+27.  S_t comes
    //     from one ballot per view slot.  Each lane ranks its views of S_t against the pixel's others (psi in
    //     LDS, the same address for the pixel's 9 lanes): a view keeps its modified importance (x2 for
    //     v_{t-1}) when fewer than k views of S_t rank above it by modified importance (larger, or equal and a
    //     lower index), a view of S_{t-1} that left the selection weighs 0.2, every other view 0; the view no
    //     other outranks by importance itself is v_t = argmax psi (ties to the lower index), found by a ballot
    uint32_t Sm = 0;
    int vt = -1;
    int vprev = -1;
    float *wgt = S.wgt + (wave * kGroups + g) * kMaxSrc;
    if (!heur) {  // uniform over the launch: every lane takes part in the ballots
        uint32_t Sprev = 0;
        if (pix_ok) {
            vprev = glob(a.st.v)[p];
            Sprev = glob(a.st.S)[p];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = row + kRows * i;
            const bool in = pix_ok && j < N && psi[j] >= 0.f;
            // bits of views j >= 32 fall off the 32-bit shift; such views do not exist (N <= 32)
            Sm |= (uint32_t)((__ballot(in) >> (kRows * grp)) & 0x1FFull) << (kRows * i);
        }
        uint32_t top = 0;  // bit i: the lane's view slot i is v_t
        if (pix_ok) {
            for (int i = 0, j = row; j < N; ++i, j += kRows) {
                const float pj = psi[j];
                if (pj >= 0.f) {  // j in S_t
                    const float mj = (j == vprev ? 2.f : 1.f) * pj;
                    int rank = 0, rpsi = 0;
                    for (uint32_t rest = Sm; rest; rest &= rest - 1u) {  // the views of S_t
                        const int q = __builtin_ctz(rest);
                        const float pq = psi[q];
                        const float mq = (q == vprev ? 2.f : 1.f) * pq;
                        rank += (mq > mj || (mq == mj && q < j)) ? 1 : 0;
                        rpsi += (pq > pj || (pq == pj && q < j)) ? 1 : 0;
                    }
                    if (rpsi == 0) top |= 1u << i;
                    wgt[j] = rank < m.k ? mj : 0.f;
                } else {
                    wgt[j] = ((Sprev >> j) & 1u) ? 0.2f : 0.f;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t bits = (uint32_t)((__ballot((top >> i) & 1u) >> (kRows * grp)) & 0x1FFull);
            if (bits) vt = kRows * i + __builtin_ctz(bits);
        }
    } else if (pix_ok) {  // heuristic selection (ablation): every view weighs 1
        for (int j = row; j < N; j += kRows) wgt[j] = 1.f;
    }
    __syncthreads();
    // S_t and v_t wait in the pixel's psi block (read no more) until the pixel is written, so that they are
    // not held in registers through the refinement
    if (pix_ok && row == 0) {
        psi[0] = __uint_as_float(Sm);
        psi[1] = __int_as_float(vt);
    }
    // the pixel's weight sum in view order; all weights 0: the plain mean over all views (uniform weights)
    float wsum = 0.f;
    if (pix_ok)
        for (int j = 0; j < N; ++j) wsum += wgt[j];
    const bool uniform = !(wsum > 0.f);
    if (uniform) wsum = (float)N;
    // made explicit for the refinement; meanwhile the pixel's lanes read 1 for every view when uniform
    if (pix_ok && uniform)
        for (int j = row; j < N; j += kRows) wgt[j] = 1.f;

    // (6) unified cost of the lane's hypothesis (Eq. 7), per row block
    for (int b = 0; b < RB; ++b) {
        const float *mc = mcol + b * WAVES * N * 64;
        const bool vb = stdp ? S.valid[b * WL + tid] != 0 : valid;
        float mfin = __builtin_inff();
        if (vb) {
            if (heur) {
                mfin = mean_k_lowest(mc + lane, 64, N, min(m.k, N));
            } else {
                float acc = 0.f;
                for (int j = 0; j < N; ++j) acc = fmaf(uniform ? 1.f : wgt[j], mc[j * 64 + lane], acc);
                mfin = acc / wsum;
            }
        }
        S.mf[b * WL + tid] = mfin;
    }
    __syncthreads();

    // (7) best hypothesis: own plane first, then region order; strictly lower wins.  Only its row is kept
    //     (its plane and cost stay in LDS): fewer registers live across the refinement's evaluations
    int brow = 8;
    if (pix_ok && !stdp) {
        const int base = wave * 64 + g * kRows;
        int br = -1;
        float bc = 0.f;
        if (S.valid[base + 8]) { br = 8; bc = S.mf[base + 8]; }
        for (int r = 0; r < 8; ++r) {
            if (!S.valid[base + r]) continue;
            const float c = S.mf[base + r];
            if (br < 0 || c < bc) { br = r; bc = c; }
        }
        brow = br < 0 ? 8 : br;  // no valid row at all (1-pixel image, no self): the own plane
    }
    int bslot = wave * 64 + g * kRows + brow;
    if (stdp && pix_ok) {
        // the own plane (row 20: block 2, lane row 2) first, then rows 0..19 in order; strictly lower wins
        const int base = wave * 64 + g * kRows;
        const int self = 2 * WL + base + 2;
        int br = -1;
        float bc = 0.f;
        if (S.valid[self]) { br = self; bc = S.mf[self]; }
        for (int i = 0; i < kStdRows; ++i) {
            const int sl = (i / 9) * WL + base + i % 9;
            if (!S.valid[sl]) continue;
            const float c = S.mf[sl];
            if (br < 0 || c < bc) { br = sl; bc = c; }
        }
        bslot = br < 0 ? self : br;
    }

    // (8) refinement (Sec. 3.3): perturbed (and, from t = 3, random) depth/normal candidates,
    //     scored with the same weights on the views that carry weight; strictly lower wins
    int n_ref = 0;
    float bcost = 0.f;  // cost of the kept hypothesis: the best row, or the candidate bcand that beat it
    int bcand = -1;
    if (m.refine) {
        const int ncand = a.t >= 3 ? 6 : 3;
        // the pixel's lanes share the set-up: lane 8 lists the active views, lane r < ncand builds candidate r
        // (candidates: (dprt, n), (d, nprt), (dprt, nprt) [, (drnd, n), (d, nrnd), (drnd, nrnd)]; the
        // perturbation draws come from stream 1, the random ones from stream 2, one draw per lane)
        if (grp < kGroups && row == 8) {
            unsigned char *act = S.act + (wave * kGroups + g) * kMaxSrc;
            int c = 0;
            if (pix_ok)
                for (int j = 0; j < N; ++j)
                    if (wgt[j] > 0.f) act[c++] = (unsigned char)j;
            S.gnw[wave * 8 + g] = c;
            S.gws[wave * 8 + g] = make_float2(ws.invW, ws.var_a);
        }
        if (pix_ok && row < ncand) {
            const float4 best = S.pl[bslot];
            const bool rnd = row >= 3;
            const int kind = rnd ? row - 3 : row;  // 0: (new depth, n), 1: (d, new normal), 2: both new
            const float2 rr = ref_ray(a.ref, x, y);
            const float dcur = plane_depth(rr, best);
            float u[4];
            philox(p, (uint64_t)a.t, rnd ? 2 : 1, m.seed, u);
            float dnew, qx, qy, qz;
            if (!rnd) {
                const float rho = ldexpf(1.f, -(a.t + 2));
                dnew = dcur + (2.f * u[0] - 1.f) * rho * (m.d_max - m.d_min);
                dnew = fminf(fmaxf(dnew, m.d_min), m.d_max);
                qx = best.x + 2.f * rho * (2.f * u[1] - 1.f);
                qy = best.y + 2.f * rho * (2.f * u[2] - 1.f);
                qz = best.z + 2.f * rho * (2.f * u[3] - 1.f);
                const float inv = 1.f / sqrtf(qx * qx + qy * qy + qz * qz);
                qx *= inv; qy *= inv; qz *= inv;
            } else {
                dnew = m.d_min + u[0] * (m.d_max - m.d_min);
                normal_from_uniforms(u[1], u[2], qx, qy, qz);
            }
            S.cand[(wave * kGroups + g) * 6 + row] =
                kind == 0 ? plane_from(rr, dnew, best.x, best.y, best.z)
                          : plane_from(rr, kind == 1 ? dcur : dnew, qx, qy, qz);
        }
        __syncthreads();
        // The (candidate, active view) pairs of a wave's 7 pixels, numbered pixel by pixel, spread over all 64
        // lanes (pixels with more active views no longer hold the wave for extra rounds); results go to the
        // pixel's area of its wave's cost-matrix LDS (7 * 6N <= 64N).  Float32 sources (the method's build): each
        // wave runs its own full rounds of 64; the pairs of the waves' last, partial rounds are pooled over the workgroup and
        // taken 64 at a time, wave w taking the w-th chunk, so that the partial rounds do not each cost a round.
        const auto ref_pair = [&](int w2, int h, int loc, int yrow) {
            const int base = w2 * kGroups + h;
            const int nwh = S.gnw[w2 * 8 + h];
            const int c = loc / nwh;
            const int j = S.act[base * kMaxSrc + (loc - c * nwh)];
            const float4 cp = S.cand[base * 6 + c];
            const float2 wsh = S.gws[w2 * 8 + h];
            const WinStats wsv = {wsh.x, wsh.y};
            const int xh = 2 * (tx * kTilePix + h) + ((yrow + a.colour) & 1);
            // only the weight and the destination stay live across the evaluation
            const float wj = S.wgt[base * kMaxSrc + j];
            float *dst = S.ms + w2 * N * 64 + (h * (6 * N) + loc);
            const PlaneQ cq = plane_q(a.ref, m, cp, xh, yrow);
            // kShort stays in the stored product (wgt > 0 on active views): counted after the loop
            const float cost = cq.ok ? ncc_cost_raw<HALF>(a.views[j], S.rw + base * kWinStride, wsv, xh, yrow, cq.q0,
                                                          cq.qu, cq.qv)
                                     : kShort;
            *dst = wj * cost;
            ++n_ref;
        };
        if constexpr (HALF || ABL) {
            // float16 sources and the ablation build: each wave takes its own pairs, its last round partial
            // (pooling measured slower in both: with many sources and candidates the waves' last rounds are
            // nearly full already, and the ablation build's code generation suffers)
            int start[kGroups + 1];
            start[0] = 0;
#pragma unroll
            for (int h = 0; h < kGroups; ++h)
                start[h + 1] = start[h] + ncand * __builtin_amdgcn_readfirstlane(S.gnw[wave * 8 + h]);
            const int yrow = __builtin_amdgcn_readfirstlane(y);
            for (int qi = lane; qi < start[kGroups]; qi += 64) {
                int h = 0;
#pragma unroll
                for (int k = 1; k < kGroups; ++k) h += qi >= start[k];
                ref_pair(wave, h, qi - start[h], yrow);
            }
        } else {
        // pair counts of every wave's pixels (wave-uniform), and the pool of the waves' partial rounds
        int tot[WAVES], pool[WAVES + 1];
        pool[0] = 0;
#pragma unroll
        for (int w2 = 0; w2 < WAVES; ++w2) {
            int acc = 0;
#pragma unroll
            for (int h = 0; h < kGroups; ++h) acc += ncand * __builtin_amdgcn_readfirstlane(S.gnw[w2 * 8 + h]);
            tot[w2] = acc;
            pool[w2 + 1] = pool[w2] + (acc & 63);
        }
        // this wave's prefix of pair counts over its pixels (wave-uniform), for the decode of its own rounds
        int start[kGroups + 1];
        start[0] = 0;
#pragma unroll
        for (int h = 0; h < kGroups; ++h)
            start[h + 1] = start[h] + ncand * __builtin_amdgcn_readfirstlane(S.gnw[wave * 8 + h]);
        const int own_full = start[kGroups] >> 6;
        // rounds of this wave: its own full rounds, then pool chunks wave, wave + WAVES, ...
        const int nchunks = (pool[WAVES] + 63) >> 6;
        const int rounds = own_full + (nchunks > wave ? (nchunks - wave + WAVES - 1) / WAVES : 0);
        for (int rd = 0; rd < rounds; ++rd) {
            int w2 = wave, h = 0, loc;
            if (rd < own_full) {
                const int qi = rd * 64 + lane;
#pragma unroll
                for (int k = 1; k < kGroups; ++k) h += qi >= start[k];
                loc = qi - start[h];
            } else {
                // pair pi of the pool belongs to wave w2, at its index (full rounds of w2) + (pi - pool[w2]);
                // the pixel h of wave w2 whose pairs hold that index, from w2's pair counts
                const int pi = (wave + (rd - own_full) * WAVES) * 64 + lane;
                if (pi >= pool[WAVES]) continue;
                int first = 0, fullw = 0;
#pragma unroll
                for (int k = 0; k < WAVES; ++k)
                    if (pi >= pool[k]) {
                        w2 = k;
                        first = pool[k];
                        fullw = tot[k] & ~63;
                    }
                const int qi = fullw + (pi - first);
                int hs = 0, acc = 0;
#pragma unroll
                for (int k = 0; k < kGroups; ++k) {
                    acc += ncand * S.gnw[w2 * 8 + k];
                    if (qi >= acc) {
                        h = k + 1;
                        hs = acc;
                    }
                }
                loc = qi - hs;
            }
            ref_pair(w2, h, loc, y0 + w2);
        }
        }
        __syncthreads();
        if (pix_ok) {
            bcost = S.mf[bslot];
            const int nw = S.gnw[wave * 8 + g];
            const int pairs = ncand * nw;
            const float *res = S.ms + wave * N * 64 + g * (6 * N);
            if (row == 0) {
                unsigned ns = 0;
                for (int i = 0; i < pairs; ++i) ns += res[i] < 0.f;
                if (ns) atomicAdd(&S.nshort[wave], ns);
            }
            for (int c = 0; c < ncand; ++c) {
                float cc;
                if (heur) {
                    cc = mean_k_lowest(res + c * nw, 1, nw, min(m.k, nw));
                } else {
                    float acc = 0.f;
                    for (int i = 0; i < nw; ++i) acc += weighted_cost(res[c * nw + i]);
                    cc = acc / wsum;
                }
                if (cc < bcost) {
                    bcost = cc;
                    bcand = c;
                }
            }
        }
    } else if (pix_ok) {
        bcost = S.mf[bslot];
    }

    // (9) write the pixel
    if (pix_ok && row == 0) {
        const float4 best = bcand < 0 ? S.pl[bslot] : S.cand[(wave * kGroups + g) * 6 + bcand];
        store_plane(a.st.planes, p, best);
        glob(a.st.cost)[p] = bcost;
        glob(a.st.S)[p] = __float_as_uint(psi[0]);
        glob(a.st.v)[p] = __float_as_int(psi[1]);
    }
    count_evals(a.counters, 1, (unsigned long long)n_prop);
    if (m.refine) count_evals(a.counters, 2, (unsigned long long)n_ref);
    // the wave's own LDS atomics are complete before this read (LDS operations of a wave are in order)
    count_evals(a.counters, 4, lane == 0 ? (unsigned long long)S.nshort[wave] : 0ull);
}

// ---------------------------------------------------------------------------
// Single-image half-pass: one workgroup per tile of the colour.
// ---------------------------------------------------------------------------
template <int HALF, int WAVES, bool ABL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ABL ? AMH_BATCH_WAVES_PER_EU : AMH_PASS_WAVES_PER_EU)))
void pass_kernel(PassArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = tile_of_block(a.n_tiles, a.order);
    if (L < 0) return;
    pass_body<HALF, WAVES, ABL>(a, L, smem, (int)threadIdx.x);
}

// ---------------------------------------------------------------------------
// Batched launch: one phase (init of a colour, or a half-pass) of many
// reference images of different sizes and view counts.  The tiles of the
// active jobs are concatenated; a workgroup finds its job by binary search in
// the prefix sums and runs the same body as the single-image kernels.  The
// workgroup that finishes the last tile of a job's last phase stamps the
// device clock (per-job completion time within the batch).
// ---------------------------------------------------------------------------
// A workgroup-uniform value read from memory, made visibly uniform (scalar registers), one dword at a time.
template <typename T>
__device__ __forceinline__ T make_uniform(const T &v) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized");
    T r;
    const int *src = reinterpret_cast<const int *>(&v);
    int *dst = reinterpret_cast<int *>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return r;
}

// Work item g of a batched phase: the active slot lo and the job-local tile (or initialisation block) L.
// Order 0: every job's items are cut into 8 contiguous bands; XCD x (workgroups round-robin over the
// XCDs) walks one band of each job in job order -- band (x + slot) mod 8 of the job at active slot `slot`,
// so that the larger bands of uneven cuts rotate over the XCDs -- and all XCDs move through the jobs
// together (one job's sources in the shared cache, neighbouring items in each XCD's L2).  xcd_pre[x][slot]
// is the prefix sum of XCD x's band sizes.  Order 1: hardware order over the concatenated items.
__device__ __forceinline__ bool batch_locate(const BatchPhaseArgs &b, int &lo, int &L) {
    if (b.order == 0) {
        const int x = blockIdx.x & 7, g = (int)(blockIdx.x >> 3);
        const int *pre = b.xcd_pre + x * (b.n_active + 1);
        if (g >= pre[b.n_active]) return false;
        int a0 = 0, a1 = b.n_active;  // pre[a0] <= g < pre[a1]
        while (a1 - a0 > 1) {
            const int mid = (a0 + a1) >> 1;
            if (pre[mid] <= g) a0 = mid;
            else a1 = mid;
        }
        lo = a0;
        const int n = b.tile_start[lo + 1] - b.tile_start[lo];
        L = (int)(((long long)n * ((x + lo) & 7)) >> 3) + (g - pre[lo]);
    } else {
        const int g = blockIdx.x;
        if (g >= b.total_tiles) return false;
        int a0 = 0, a1 = b.n_active;  // tile_start[a0] <= g < tile_start[a1]
        while (a1 - a0 > 1) {
            const int mid = (a0 + a1) >> 1;
            if (b.tile_start[mid] <= g) a0 = mid;
            else a1 = mid;
        }
        lo = a0;
        L = g - b.tile_start[lo];
    }
    return true;
}

// The single-image arguments of job J in a batched phase, in scalar registers (the job's arguments are the
// same for the whole workgroup; the source table as an offset from the argument's pointer, so that the
// per-view constants are read like the single-image kernels read theirs: scalar loads)
__device__ __forceinline__ PassArgs batch_pass_args(const BatchPhaseArgs &b, const BatchJobDev &J, int waves) {
    PassArgs a;
    a.ref = J.ref;
    a.n_src = J.n_src;
    a.m = b.m;
    a.st = J.st;
    a.t = b.t;
    a.colour = b.colour;
    a.tiles_x = J.tiles_x;
    a.n_tiles = J.n_tiles;
    a.counters = b.counters;
    a.order = b.order;
    a.waves = waves;
    a.prop = J.prop;
    a.prop_w = J.prop_w;
    a.prop_s = kCell;
    a.conf_min = b.conf_min;
    a = make_uniform(a);
    a.views = b.views + __builtin_amdgcn_readfirstlane(J.view_off);
    return a;
}

// the job's completion time: stamped by the last work item of its last phase
__device__ __forceinline__ void batch_stamp(const BatchPhaseArgs &b, int lo, int j, long long items) {
    if (b.is_last[lo]) {
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            if (atomicAdd(&b.tiles_done[j], 1ull) == (unsigned long long)(items - 1)) b.job_end[j] = wall_clock64();
        }
    }
}

// Batched half-pass: one tile per workgroup.
template <int HALF, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AMH_PASS_WAVES_PER_EU)))
void batch_kernel(BatchPhaseArgs b) {
    extern __shared__ __align__(16) unsigned char smem[];
    int lo, L;
    if (!batch_locate(b, lo, L)) return;
    const int j = b.job_of[lo];
    const BatchJobDev &J = b.jobs[j];
    const PassArgs a = batch_pass_args(b, J, WAVES);
    pass_body<HALF, WAVES>(a, __builtin_amdgcn_readfirstlane(L), smem, (int)threadIdx.x);
    batch_stamp(b, lo, j, J.n_tiles);
}

// Batched initialisation: one initialisation block (kInitBlock pixels of the colour) per workgroup, the body
// of the single-image kernel, so that a job's initial state is the same bits either way.
template <int HALF>
__global__ __launch_bounds__(2 * kInitBlock) __attribute__((amdgpu_waves_per_eu(AMH_INIT_WAVES_PER_EU))) void
batch_init_kernel(BatchPhaseArgs b) {
    extern __shared__ __align__(16) float cst[];  // [max n_src][kInitBlock]
    __shared__ unsigned nshort;
    int lo, L;
    if (!batch_locate(b, lo, L)) return;
    const int j = b.job_of[lo];
    const BatchJobDev &J = b.jobs[j];
    const PassArgs a = batch_pass_args(b, J, 4);
    init_pair_body<HALF>(a, __builtin_amdgcn_readfirstlane(L), cst, &nshort);
    batch_stamp(b, lo, j, J.n_iblocks);
}

// ---------------------------------------------------------------------------
// Persistent batched launch (see PersistArgs): one kernel runs every
// half-pass of every job (the two initialisation phases before it are
// ordinary batched launches).
// ---------------------------------------------------------------------------
// Grid barrier between phases: every thread releases its writes at device scope, the workgroup counts its
// arrival, waits (bounded) until `target` workgroups arrived, and acquires.  False when a wait ran out.
__device__ __forceinline__ bool grid_barrier(const PersistArgs *P, unsigned target, int *s_ok) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(P->arrived, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t0 = wall_clock64();
        int ok = 1;
        while (__hip_atomic_load(P->arrived, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(P->fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                wall_clock64() - t0 > P->spin_limit) {
                __hip_atomic_fetch_or(P->fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        *s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *s_ok != 0;
}

// The launch's arguments live in device memory and are re-read around every tile through a pointer the
// compiler cannot treat as loop-invariant, so that none of them occupies registers during the tile's body.
__device__ __forceinline__ const PersistArgs *opaque(const PersistArgs *p) {
    asm volatile("" : "+s"(p));
    return p;
}

template <int HALF, int WAVES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AMH_PASS_WAVES_PER_EU)))
void persist_kernel(const PersistArgs *__restrict__ Pg) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item, s_ok;
    const int x = blockIdx.x & 7;
    if (Pg->probe) {  // how many workgroups of this kernel are resident at once
        if (threadIdx.x == 0) {
            unsigned *in = Pg->next, *out = Pg->next + 1, *peak = Pg->next + 2;
            __hip_atomic_fetch_add(in, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long t0 = wall_clock64();
            unsigned most = 0;
            for (;;) {
                const unsigned a = __hip_atomic_load(in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned b = __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                most = max(most, a - b);
                if (most >= gridDim.x || wall_clock64() - t0 > Pg->probe_ticks) break;
                __builtin_amdgcn_s_sleep(4);
            }
            __hip_atomic_fetch_max(peak, most, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    const int n_phases = __builtin_amdgcn_readfirstlane(Pg->n_phases);
    for (int ph = 0; ph < n_phases; ++ph) {
        for (;;) {
            const PersistArgs *P = opaque(Pg);
            if (threadIdx.x == 0) s_item = (int)atomicAdd(&P->next[ph * 8 + x], 1u);
            __syncthreads();
            const int g = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
            const PersistPhase Q = make_uniform(P->phases[ph]);
            const int *pre = Q.xcd_pre + x * (Q.n_active + 1);
            if (g >= __builtin_amdgcn_readfirstlane(pre[Q.n_active])) break;
            // the g-th tile of this XCD's queue: band (x + slot) mod 8 of the job at active slot `slot`
            int a0 = 0, a1 = Q.n_active;  // pre[a0] <= g < pre[a1]
            while (a1 - a0 > 1) {
                const int mid = (a0 + a1) >> 1;
                if (pre[mid] <= g) a0 = mid;
                else a1 = mid;
            }
            const int lo = __builtin_amdgcn_readfirstlane(a0);
            const int n = Q.tile_start[lo + 1] - Q.tile_start[lo];
            const int L = __builtin_amdgcn_readfirstlane((int)(((long long)n * ((x + lo) & 7)) >> 3) + (g - pre[lo]));
            const int j = __builtin_amdgcn_readfirstlane(Q.job_of[lo]);
            const BatchJobDev &J = P->jobs[j];
            PassArgs a;
            a.ref = J.ref;
            a.n_src = J.n_src;
            a.m = Q.m;
            a.st = J.st;
            a.t = Q.t;
            a.colour = Q.colour;
            a.tiles_x = J.tiles_x;
            a.n_tiles = J.n_tiles;
            a.counters = P->counters;
            a.order = 0;
            a.waves = WAVES;
            a.prop = J.prop;
            a.prop_w = J.prop_w;
            a.prop_s = kCell;
            a.conf_min = P->conf_min;
            a = make_uniform(a);
            a.views = P->views + __builtin_amdgcn_readfirstlane(J.view_off);
            int tid = (int)threadIdx.x;
            asm volatile("" : "+v"(tid));
            pass_body<HALF, WAVES>(a, L, smem, tid);
            // per-job completion stamp of the job's last half-pass
            const PersistArgs *P2 = opaque(Pg);
            if (P2->phases[ph].is_last[lo]) {
                __syncthreads();
                if (threadIdx.x == 0) {
                    __threadfence();
                    if (atomicAdd(&P2->tiles_done[j], 1ull) == (unsigned long long)(P2->jobs[j].n_tiles - 1))
                        P2->job_end[j] = wall_clock64();
                }
            }
        }
        if (ph + 1 < n_phases && !grid_barrier(opaque(Pg), (unsigned)(ph + 1) * gridDim.x, &s_ok)) return;
    }
}

__global__ void stamp_kernel(unsigned long long *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = wall_clock64();
}

// ---------------------------------------------------------------------------
// Fixed hypotheses: one thread per (query, view).
// ---------------------------------------------------------------------------
template <int HALF>
__global__ __launch_bounds__(64) void score_kernel(ScoreArgs a) {
    __shared__ __align__(16) float2 rwbuf[64 * kWinStride];
    const int gid = blockIdx.x * 64 + threadIdx.x;
    const int total = a.Q * a.n_src;
    if (gid >= total) return;  // no barrier in this kernel
    const int qi = gid / a.n_src, j = gid - qi * a.n_src;
    const int2 px = a.pix[qi];
    const float4 pl = a.planes[qi];
    float2 *rw = rwbuf + threadIdx.x * kWinStride;
    GlobalReader rd{&a.ref, px.x, px.y};
    const WinStats ws = build_window(rd, a.m, rw, 0, 1);
    const PlaneQ q = plane_q(a.ref, a.m, pl, px.x, px.y);
    a.costs[gid] = q.ok ? ncc_cost<HALF>(a.views[j], rw, ws, px.x, px.y, q.q0, q.qu, q.qv) : 2.f;
}

// ---------------------------------------------------------------------------
// Plane-sweep input of the proposal network, on a grid of 8 ceil(H/32) x
// 8 ceil(W/32) cells of 4 x 4 pixels.  A workgroup of 64 lanes takes 16
// cells x 4 consecutive sweep planes: lane (cell, k) scores planes k, k + 4,
// k + 8, ... of its cell on every source in turn, so at any instruction the
// whole wave gathers from one source, and the 4 lanes of a cell warp to
// positions ~2 px apart (consecutive planes) that share texel lines.  A lane
// aggregates its plane's costs (mean of the min(2, n) lowest), keeps its best
// plane and the best aggregate of every coarse bin; the 4 lanes of a cell
// merge these with shuffles at the end (ties: lowest plane index).  The
// window of the cell's sample pixel (4j + 2, 4i + 2; clamped to the image) is
// built once per cell.
// Channels: normalised mean and deviation of the cell's 4 x 4 reference
// pixels, winning plane position, 1 - its cost, 1 - best cost per coarse bin;
// the winner's inverse depth is also written in fp32 (the depth base of the
// network's refinement head).
// ---------------------------------------------------------------------------
template <int HALF>
__global__ __launch_bounds__(64) void sweep_kernel(SweepArgs a) {
    // one window block per cell, written a quarter by each of its 4 lanes
    __shared__ __align__(16) float2 rwbuf[16 * kWinStride];
    const int lane = threadIdx.x, cl = lane >> 2, k = lane & 3;
    const int n_cells = a.h4 * a.w4;
    const int cell = blockIdx.x * 16 + cl;
    const bool cell_ok = cell < n_cells;
    const int ci = cell_ok ? cell / a.w4 : 0, cj = cell_ok ? cell - ci * a.w4 : 0;
    // sample pixel, clamped to the image (cells past the right or bottom edge repeat the edge)
    const int x = min(kCell * cj + kCell / 2, a.ref.W - 1), y = min(kCell * ci + kCell / 2, a.ref.H - 1);
    float2 *rw = rwbuf + cl * kWinStride;
    WinStats ws = {1.f, 0.f};
    if (cell_ok) {
        GlobalReader rd{&a.ref, x, y};
        ws = build_window(rd, a.m, rw, k, 4);
    }
    __syncthreads();
    const float inf = __builtin_inff();
    const int n = a.n_net;
    float best = inf, coarse[kSweepCoarse];
    int best_i = 0x7fffffff;
#pragma unroll
    for (int c = 0; c < kSweepCoarse; ++c) coarse[c] = inf;
    const int D = kSweepCoarse * a.sub;  // a multiple of 4
    if (cell_ok) {
        for (int i = k; i < D; i += 4) {
            const float qi = a.q_far + ((float)i + 0.5f) * a.q_step;
            const PlaneQ q = plane_q(a.ref, a.m, make_float4(0.f, 0.f, -1.f, 1.f / qi), x, y);
            float m1 = inf, m2 = inf;  // two lowest costs over the sources
            for (int j = 0; j < n; ++j) {
                const float c = q.ok ? ncc_cost<HALF>(a.views[j], rw, ws, x, y, q.q0, q.qu, q.qv) : 2.f;
                m2 = fminf(m2, fmaxf(m1, c));
                m1 = fminf(m1, c);
            }
            const float agg = n >= kSweepK ? 0.5f * (m1 + m2) : m1;
            if (agg < best) {
                best = agg;
                best_i = i;
            }
            const int cb = i / a.sub;
#pragma unroll
            for (int cc = 0; cc < kSweepCoarse; ++cc)
                if (cc == cb) coarse[cc] = fminf(coarse[cc], agg);
        }
    }
    count_evals(a.counters, 0, cell_ok ? (unsigned long long)(D / 4) * n : 0ull);
    // merge the 4 lanes of the cell (lanes 4 cl .. 4 cl + 3)
#pragma unroll
    for (int off = 1; off <= 2; off <<= 1) {
        const float ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(best_i, off, 64);
        if (ob < best || (ob == best && oi < best_i)) {
            best = ob;
            best_i = oi;
        }
#pragma unroll
        for (int cc = 0; cc < kSweepCoarse; ++cc) coarse[cc] = fminf(coarse[cc], __shfl_xor(coarse[cc], off, 64));
    }
    if (!cell_ok) return;  // no barrier follows
    unsigned short *out = a.feats + (size_t)cell * 16;
    if (k == 0) {
        // the cell's 4 x 4 pixels, coordinates clamped to the image
        float px[kCell * kCell];
        for (int yy = 0; yy < kCell; ++yy)
            for (int xx = 0; xx < kCell; ++xx)
                px[yy * kCell + xx] = a.ref.img[(size_t)min(kCell * ci + yy, a.ref.H - 1) * a.ref.W +
                                                min(kCell * cj + xx, a.ref.W - 1)];
        float mu = 0.f;
        for (int e = 0; e < kCell * kCell; ++e) mu += px[e];
        mu *= 1.f / (kCell * kCell);
        float var = 0.f;
        for (int e = 0; e < kCell * kCell; ++e) {
            const float dlt = px[e] - mu;
            var = fmaf(dlt, dlt, var);
        }
        out[0] = f2bf((mu - 127.5f) * (1.f / 64.f));
        out[1] = f2bf(__builtin_sqrtf(var * (1.f / (kCell * kCell))) * (1.f / 32.f));
        out[2] = f2bf(2.f * ((float)best_i + 0.5f) / (float)D - 1.f);
        out[3] = f2bf(1.f - best);
        if (a.q_ref) a.q_ref[cell] = a.q_far + ((float)best_i + 0.5f) * a.q_step;
    } else {
        // lanes 1..3 write 4 coarse channels each
#pragma unroll
        for (int cc = 0; cc < kSweepCoarse; ++cc)
            if (cc / 4 == k - 1) out[4 + cc] = f2bf(1.f - coarse[cc]);
    }
}

// ---------------------------------------------------------------------------
// Layout kernels
// ---------------------------------------------------------------------------
__global__ void convert_kernel(const void *src, int dtype, int64_t pitch, int W, int H, float *dst) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= W || y >= H) return;
    float v;
    if (dtype == 0) v = reinterpret_cast<const float *>(src)[(size_t)y * pitch + x];
    else v = __half2float(reinterpret_cast<const __half *>(src)[(size_t)y * pitch + x]);
    dst[(size_t)y * W + x] = v;
}

__global__ void pack_quads_kernel(const float *img, int W, int H, void *quads, int half) {
    const int xx = blockIdx.x * blockDim.x + threadIdx.x, yy = blockIdx.y;  // 0..W+1+2P, 0..H+2P
    if (xx > W + 1 + 2 * kQuadPad || yy > H + 2 * kQuadPad) return;
    const int x = min(max(xx - 1 - kQuadPad, 0), W - 1);
    const int y0 = min(max(yy - 1 - kQuadPad, 0), H - 1), y1 = min(max(yy - kQuadPad, 0), H - 1);
    const float a = img[(size_t)y0 * W + x], c = img[(size_t)y1 * W + x];
    const size_t i = (size_t)yy * (W + 2 + 2 * kQuadPad) + xx;
    if (!half) {
        // the difference rounded once from its exact double value
        reinterpret_cast<float2 *>(quads)[i] = make_float2(a, (float)((double)c - (double)a));
    } else {
        reinterpret_cast<__half2 *>(quads)[i] = __floats2half2_rn(a, c);
    }
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// per-pixel hypotheses (depth, normal, confidence) interleaved as the initialisation reads predictions
__global__ void pack_hypotheses_kernel(const float *depth, const float *normal, const float *conf, int64_t n,
                                       float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float *o = out + i * 5;
        o[0] = depth[i];
        o[1] = normal[3 * i];
        o[2] = normal[3 * i + 1];
        o[3] = normal[3 * i + 2];
        o[4] = conf ? conf[i] : 1.f;
    }
}

__global__ void outputs_kernel(RefDev ref, StateDev st, float *depth, float *normal, float *cost) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= ref.W || y >= ref.H) return;
    const size_t p = (size_t)y * ref.W + x;
    const float4 pl = st.planes[p];
    if (depth) {
        const double rx = fma(ref.kinv_a, (double)x, fma(ref.kinv_b, (double)y, ref.kinv_c));
        const double ry = fma(ref.kinv_e, (double)y, ref.kinv_f);
        depth[p] = (float)(-(double)pl.w / ((double)pl.x * rx + (double)pl.y * ry + (double)pl.z));
    }
    if (normal) {
        normal[3 * p] = pl.x;
        normal[3 * p + 1] = pl.y;
        normal[3 * p + 2] = pl.z;
    }
    if (cost) cost[p] = st.cost[p];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Clears an error left by an earlier, unrelated runtime call, so that the
// hipGetLastError() after the launch reports the launch itself.
#define AMH_LAUNCH(...)                  \
    do {                                 \
        (void)hipGetLastError();         \
        hipLaunchKernelGGL(__VA_ARGS__); \
    } while (0)

hipError_t launch_pack_hypotheses(const float *depth, const float *normal, const float *conf, int64_t n, float *out,
                                  hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    AMH_LAUNCH(pack_hypotheses_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, depth, normal,
               conf, n, out);
    return hipGetLastError();
}

hipError_t launch_convert_to_f32(const void *src, int src_dtype, int64_t pitch, int W, int H, float *dst,
                                 hipStream_t s) {
    dim3 grid((W + 255) / 256, H);
    AMH_LAUNCH(convert_kernel, grid, dim3(256), 0, s, src, src_dtype, pitch, W, H, dst);
    return hipGetLastError();
}

hipError_t launch_pack_quads(const float *img, int W, int H, void *quads, int half, hipStream_t s) {
    dim3 grid((W + 2 + 2 * kQuadPad + 255) / 256, H + 1 + 2 * kQuadPad);
    AMH_LAUNCH(pack_quads_kernel, grid, dim3(256), 0, s, img, W, H, quads, half);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s) {
    AMH_LAUNCH(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

static inline int grid_for(int n_tiles) { return ((n_tiles + 7) / 8) * 8; }

hipError_t launch_init(const PassArgs &a, int half, hipStream_t s) {
    const dim3 grid((unsigned)(8 * ((init_blocks(a.ref.W, a.ref.H) + 7) / 8)));
    const size_t lds = sizeof(float) * kInitBlock * a.n_src;
    if (half) AMH_LAUNCH(init_pair_kernel<1>, grid, dim3(2 * kInitBlock), lds, s, a);
    else AMH_LAUNCH(init_pair_kernel<0>, grid, dim3(2 * kInitBlock), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_pass(const PassArgs &a, int half, hipStream_t s) {
    const size_t lds = pass_lds_bytes(a.n_src, a.waves, a.m.sym_prop == 2 ? 3 : 1);
    const dim3 grid(grid_for(a.n_tiles)), block(64 * a.waves);
    const bool abl = a.m.sym_prop || a.m.heuristic;
    if (a.waves == 2) {
        if (abl) {
            if (half) AMH_LAUNCH((pass_kernel<1, 2, true>), grid, block, lds, s, a);
            else AMH_LAUNCH((pass_kernel<0, 2, true>), grid, block, lds, s, a);
        } else {
            if (half) AMH_LAUNCH((pass_kernel<1, 2, false>), grid, block, lds, s, a);
            else AMH_LAUNCH((pass_kernel<0, 2, false>), grid, block, lds, s, a);
        }
    } else if (a.waves == 4) {
        if (abl) {
            if (half) AMH_LAUNCH((pass_kernel<1, 4, true>), grid, block, lds, s, a);
            else AMH_LAUNCH((pass_kernel<0, 4, true>), grid, block, lds, s, a);
        } else {
            if (half) AMH_LAUNCH((pass_kernel<1, 4, false>), grid, block, lds, s, a);
            else AMH_LAUNCH((pass_kernel<0, 4, false>), grid, block, lds, s, a);
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch(const BatchPhaseArgs &b, int half, int max_src, hipStream_t s) {
    if (b.total_tiles == 0) return hipSuccess;
    const dim3 grid(b.grid);
    if (b.kind == 0) {
        const size_t lds = sizeof(float) * kInitBlock * max_src;
        if (half) AMH_LAUNCH(batch_init_kernel<1>, grid, dim3(2 * kInitBlock), lds, s, b);
        else AMH_LAUNCH(batch_init_kernel<0>, grid, dim3(2 * kInitBlock), lds, s, b);
        return hipGetLastError();
    }
    const size_t lds = pass_lds_bytes(max_src, b.waves);
    const dim3 block(64 * b.waves);
    if (b.waves == 2) {
        if (half) AMH_LAUNCH((batch_kernel<1, 2>), grid, block, lds, s, b);
        else AMH_LAUNCH((batch_kernel<0, 2>), grid, block, lds, s, b);
    } else if (b.waves == 4) {
        if (half) AMH_LAUNCH((batch_kernel<1, 4>), grid, block, lds, s, b);
        else AMH_LAUNCH((batch_kernel<0, 4>), grid, block, lds, s, b);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t persist_lds_bytes(int max_src, int waves) { return pass_lds_bytes(max_src, waves); }

int persist_blocks_per_cu(int half, int waves, int max_src) {
    const size_t lds = persist_lds_bytes(max_src, waves);
    int nb = 0;
    hipError_t e;
    if (waves == 2) e = half ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel<1, 2>, 128, lds)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel<0, 2>, 128, lds);
    else e = half ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel<1, 4>, 256, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel<0, 4>, 256, lds);
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_persist(const PersistArgs *a, int half, int waves, int max_src, int grid, hipStream_t s) {
    const size_t lds = persist_lds_bytes(max_src, waves);
    const dim3 g(grid), block(64 * waves);
    if (waves == 2) {
        if (half) AMH_LAUNCH((persist_kernel<1, 2>), g, block, lds, s, a);
        else AMH_LAUNCH((persist_kernel<0, 2>), g, block, lds, s, a);
    } else if (waves == 4) {
        if (half) AMH_LAUNCH((persist_kernel<1, 4>), g, block, lds, s, a);
        else AMH_LAUNCH((persist_kernel<0, 4>), g, block, lds, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stamp(unsigned long long *p, hipStream_t s) {
    AMH_LAUNCH(stamp_kernel, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs &a, int half, hipStream_t s) {
    const int n_cells = a.h4 * a.w4;
    if (n_cells == 0) return hipSuccess;
    dim3 grid((n_cells + 15) / 16);
    if (half) AMH_LAUNCH(sweep_kernel<1>, grid, dim3(64), 0, s, a);
    else AMH_LAUNCH(sweep_kernel<0>, grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_score(const ScoreArgs &a, int half, hipStream_t s) {
    const int total = a.Q * a.n_src;
    if (total == 0) return hipSuccess;
    dim3 grid((total + 63) / 64);
    if (half) AMH_LAUNCH(score_kernel<1>, grid, dim3(64), 0, s, a);
    else AMH_LAUNCH(score_kernel<0>, grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_outputs(const RefDev &ref, const StateDev &st, float *depth, float *normal, float *cost,
                          hipStream_t s) {
    dim3 grid((ref.W + 255) / 256, ref.H);
    AMH_LAUNCH(outputs_kernel, grid, dim3(256), 0, s, ref, st, depth, normal, cost);
    return hipGetLastError();
}

}  // namespace amh
