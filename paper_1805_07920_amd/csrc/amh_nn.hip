// gfx950 kernels of the proposal network: a 4-level convolutional
// encoder-decoder over bf16 NHWC activations with fp32 accumulation on the
// matrix cores, its backward pass, the training loss and Adam.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16:
//   forward / input gradient: rows = 16 pixels, columns = 16 output channels,
//     K = taps x input channels (padded to a multiple of 32 with zero weights);
//     each lane feeds 8 consecutive channels of one tap of one pixel, so an A
//     operand is one 16-byte load;
//   weight gradient: rows = 16 output channels, columns = 16 (tap, channel)
//     pairs, K = pixels, split over workgroups into partial sums that a second
//     kernel adds in a fixed order (deterministic, no atomics).
// The input gradient is a forward convolution of the output gradient with the
// weights transposed and the taps mirrored; the ReLU of the layer below is
// applied in its epilogue as a mask.  All channel counts are multiples of 16.
#include <hip/hip_runtime.h>

#include "amh_bf16.h"
#include "amh_nn.h"

namespace amh {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

#define NN_LAUNCH(...)                   \
    do {                                 \
        (void)hipGetLastError();         \
        hipLaunchKernelGGL(__VA_ARGS__); \
    } while (0)

// ---------------------------------------------------------------------------
// convolution (forward, and input gradient with transposed weights)
// ---------------------------------------------------------------------------
template <int NT, int OUT_F32>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = a.n * a.h * a.w;
    const int p0 = (blockIdx.x * 4 + wave) * 16;
    if (p0 >= P) return;  // no barriers in this kernel
    const int row = lane & 15, grp = lane >> 4;
    const int p = p0 + row;
    const bool pv = p < P;
    int b = 0, y = 0, x = 0;
    if (pv) {
        x = p % a.w;
        const int t = p / a.w;
        y = t % a.h;
        b = t / a.h;
    }
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r = a.ks >> 1;
    const int K = a.ks * a.ks * a.cin;
    const bf16_t *wrow = a.wgt + (size_t)row * a.kpad;
    const size_t wstride = (size_t)16 * a.kpad;
    for (int k0 = 0; k0 < a.kpad; k0 += 32) {
        const int k = k0 + grp * 8;
        u32x4 av = {0u, 0u, 0u, 0u};
        if (pv && k < K) {
            const int tap = k / a.cin, c = k - tap * a.cin;
            const int ty = tap / a.ks;
            const int yy = y + ty - r, xx = x + (tap - ty * a.ks) - r;
            if (yy >= 0 && yy < a.h && xx >= 0 && xx < a.w)
                av = *reinterpret_cast<const u32x4 *>(a.x + ((size_t)(b * a.h + yy) * a.w + xx) * a.cin + c);
        }
        const bf16x8 A = __builtin_bit_cast(bf16x8, av);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const u32x4 bv = *reinterpret_cast<const u32x4 *>(wrow + t * wstride + k);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
        }
    }
    // acc[t][i] holds output (pixel p0 + 4 grp + i, channel 16 t + row)
    const int C = NT * 16;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + row;
        const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pp = p0 + 4 * grp + i;
            if (pp >= P) continue;
            float v = acc[t][i] + bias;
            if (a.relu) v = fmaxf(v, 0.f);
            const size_t o = (size_t)pp * C + co;
            if (a.mask && !(bf2f(a.mask[o]) > 0.f)) v = 0.f;
            if (OUT_F32) reinterpret_cast<float *>(a.y)[o] = v;
            else reinterpret_cast<bf16_t *>(a.y)[o] = f2bf(v);
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: part[s][co][k] = sum over the pixels of split s of
// g[p][co] * x[p + offset(tap)][c], k = tap * cin + c;  bpart[s][co] = sum g[p][co]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s = blockIdx.x;
    const int j0 = (blockIdx.y * 4 + wave) * 16;
    const int co0 = blockIdx.z * 16;
    if (j0 >= a.kpad) return;  // no barriers in this kernel
    const int P = a.n * a.h * a.w;
    const int beg = s * a.chunk, end = min(P, beg + a.chunk);
    const int i16 = lane & 15, grp = lane >> 4;
    const int co = co0 + i16;
    const int j = j0 + i16;
    const int K = a.ks * a.ks * a.cin;
    const int r = a.ks >> 1;
    const bool jv = j < K;
    int c = 0, dy = 0, dx = 0;
    if (jv) {
        const int tap = j / a.cin;
        c = j - tap * a.cin;
        dy = tap / a.ks - r;
        dx = tap - (tap / a.ks) * a.ks - r;
    }
    const bool do_bias = blockIdx.y == 0 && wave == 0;
    float bsum = 0.f;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int pb = beg; pb < end; pb += 32) {
        const int q0 = pb + grp * 8;
        int x = 0, y = 0, b = 0;
        if (q0 < end) {
            x = q0 % a.w;
            const int t = q0 / a.w;
            y = t % a.h;
            b = t / a.h;
        }
        bf16_t av[8], bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int q = q0 + e;
            bf16_t ga = 0, xb = 0;
            if (q < end) {
                ga = a.g[(size_t)q * a.cout_pad + co];
                const int yy = y + dy, xx = x + dx;
                if (jv && yy >= 0 && yy < a.h && xx >= 0 && xx < a.w)
                    xb = a.x[((size_t)(b * a.h + yy) * a.w + xx) * a.cin + c];
            }
            av[e] = ga;
            bv[e] = xb;
            if (do_bias) bsum += bf2f(ga);
            if (++x == a.w) {
                x = 0;
                if (++y == a.h) {
                    y = 0;
                    ++b;
                }
            }
        }
        u32x4 au, bu;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            au[e] = (uint32_t)av[2 * e] | ((uint32_t)av[2 * e + 1] << 16);
            bu[e] = (uint32_t)bv[2 * e] | ((uint32_t)bv[2 * e + 1] << 16);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, au), __builtin_bit_cast(bf16x8, bu),
                                                      acc, 0, 0, 0);
    }
    // acc[i] = dW[co0 + 4 grp + i][j0 + i16]
    float *dst = a.part + (size_t)s * a.cout_pad * a.kpad;
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[(size_t)(co0 + 4 * grp + i) * a.kpad + j0 + i16] = acc[i];
    if (do_bias) {
        bsum += __shfl_xor(bsum, 16, 64);
        bsum += __shfl_xor(bsum, 32, 64);
        if (grp == 0) a.bpart[(size_t)s * a.cout_pad + co] = bsum;
    }
}

// grad[e] = sum_s part[s][e] for e < n_w (weights), then the biases
__global__ void wgrad_reduce_kernel(const float *part, const float *bpart, int splits, int n_w, int n_b, float *gw,
                                    float *gb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n_w) {
        float s = 0.f;
        for (int k = 0; k < splits; ++k) s += part[(size_t)k * n_w + e];
        gw[e] = s;
    } else if (e < n_w + n_b) {
        const int o = e - n_w;
        float s = 0.f;
        for (int k = 0; k < splits; ++k) s += bpart[(size_t)k * n_b + o];
        gb[o] = s;
    }
}

// W'[ci][tap' * cout_pad + co] = W[co][(ks^2 - 1 - tap') * cin + ci]   (zero beyond ks^2 * cout_pad)
__global__ void transpose_w_kernel(const bf16_t *w, int cin, int cout_pad, int kpad, int ks, bf16_t *wt,
                                   int kpad_t) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cin * kpad_t) return;
    const int ci = e / kpad_t, k = e - ci * kpad_t;
    bf16_t v = 0;
    if (k < ks * ks * cout_pad) {
        const int tp = k / cout_pad, co = k - tp * cout_pad;
        const int tap = ks * ks - 1 - tp;
        v = w[(size_t)co * kpad + tap * cin + ci];
    }
    wt[e] = v;
}

// ---------------------------------------------------------------------------
// pooling, upsampling + concatenation, and their gradients (8 channels/thread)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load8(const bf16_t *p, float v[8]) {
    const u32x4 u = *reinterpret_cast<const u32x4 *>(p);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[2 * e] = bf2f((bf16_t)(u[e] & 0xffffu));
        v[2 * e + 1] = bf2f((bf16_t)(u[e] >> 16));
    }
}

__device__ __forceinline__ void store8(bf16_t *p, const float v[8]) {
    u32x4 u;
#pragma unroll
    for (int e = 0; e < 4; ++e) u[e] = (uint32_t)f2bf(v[2 * e]) | ((uint32_t)f2bf(v[2 * e + 1]) << 16);
    *reinterpret_cast<u32x4 *>(p) = u;
}

// y[b][i][j] = mean of x over the 2 x 2 block (h, w: output size)
__global__ void pool_kernel(const bf16_t *x, int n, int h, int w, int C, bf16_t *y) {
    const int C8 = C / 8;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * h * w * C8) return;
    const int c = (e % C8) * 8, q = e / C8;
    const int j = q % w, t = q / w, i = t % h, b = t / h;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0}, v[8];
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            load8(x + ((size_t)(b * 2 * h + 2 * i + dy) * 2 * w + 2 * j + dx) * C + c, v);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += v[k];
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] *= 0.25f;
    store8(y + (size_t)q * C + c, s);
}

// out[b][y][x] = [low[b][y/2][x/2] (C1 channels), skip[b][y][x] (C2)]  (h, w: output size)
__global__ void upcat_kernel(const bf16_t *low, int C1, const bf16_t *skip, int C2, int n, int h, int w, bf16_t *out) {
    const int C = C1 + C2, C8 = C / 8;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * h * w * C8) return;
    const int c = (e % C8) * 8, q = e / C8;
    const int x = q % w, t = q / w, y = t % h, b = t / h;
    const bf16_t *src = c < C1 ? low + ((size_t)(b * (h / 2) + y / 2) * (w / 2) + x / 2) * C1 + c
                               : skip + (size_t)q * C2 + (c - C1);
    *reinterpret_cast<u32x4 *>(out + (size_t)q * C + c) = *reinterpret_cast<const u32x4 *>(src);
}

// gradient of an encoder output e that feeds both the pooling below and the
// decoder's concatenation:  g = (pool_grad(dp) + dcat[.., off + c]) * (e > 0)   (h, w: e's size)
__global__ void enc_grad_kernel(const bf16_t *dp, const bf16_t *dcat, int Ccat, int off, const bf16_t *e_act, int n,
                                int h, int w, int C, bf16_t *g) {
    const int C8 = C / 8;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * h * w * C8) return;
    const int c = (e % C8) * 8, q = e / C8;
    const int x = q % w, t = q / w, y = t % h, b = t / h;
    float a[8], d[8], m[8];
    load8(dp + ((size_t)(b * (h / 2) + y / 2) * (w / 2) + x / 2) * C + c, a);
    load8(dcat + (size_t)q * Ccat + off + c, d);
    load8(e_act + (size_t)q * C + c, m);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = m[k] > 0.f ? fmaf(0.25f, a[k], d[k]) : 0.f;
    store8(g + (size_t)q * C + c, a);
}

// gradient of a low-resolution map upsampled into channels [0, C1) of a
// concatenation:  g = (sum over the 2 x 2 block of dcat) * (act > 0)   (h, w: low size)
__global__ void up_grad_kernel(const bf16_t *dcat, int Ccat, const bf16_t *act, int n, int h, int w, int C1,
                               bf16_t *g) {
    const int C8 = C1 / 8;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * h * w * C8) return;
    const int c = (e % C8) * 8, q = e / C8;
    const int j = q % w, t = q / w, i = t % h, b = t / h;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0}, v[8], m[8];
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            load8(dcat + ((size_t)(b * 2 * h + 2 * i + dy) * 2 * w + 2 * j + dx) * Ccat + c, v);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += v[k];
        }
    load8(act + (size_t)q * C1 + c, m);
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = m[k] > 0.f ? s[k] : 0.f;
    store8(g + (size_t)q * C1 + c, s);
}

// ---------------------------------------------------------------------------
// head decoding, loss and its gradient
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + __expf(-z)); }

// depth head: q = clamp(q_ref + R tanh(z0), q_far, q_near); returns q and dq/dz0 (0 where clamped)
__device__ __forceinline__ float head_q(float z0, float q_ref, const DepthHead &dh, float &dq) {
    const float th = tanhf(z0);
    const float u = fmaf(dh.R, th, q_ref);
    const bool inside = u > dh.q_far && u < dh.q_near;
    dq = inside ? dh.R * (1.f - th * th) : 0.f;
    return fminf(fmaxf(u, dh.q_far), dh.q_near);
}

// z: [P][16] head output (channels 0..4 used) -> out [P][5]: depth, unit normal, confidence
__global__ void decode_kernel(const float *z, const float *q_ref, int P, DepthHead dh, float *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float *zp = z + (size_t)p * 16;
    const float nx = zp[1], ny = zp[2], nz = zp[3];
    const float inv = 1.f / __builtin_sqrtf(nx * nx + ny * ny + nz * nz);
    float dq;
    float *o = out + (size_t)p * 5;
    o[0] = 1.f / head_q(zp[0], q_ref[p], dh, dq);
    o[1] = nx * inv;
    o[2] = ny * inv;
    o[3] = nz * inv;
    o[4] = sigmoidf(zp[4]);
}

// per pixel: w (|s - t_d| + 1 - n_hat . n_t) + softplus(z4) - t_c z4, and dL/dz / P
__global__ __launch_bounds__(256) void loss_kernel(const float *z, const float *q_ref, const float *target, int P,
                                                   DepthHead dh, bf16_t *dz, float *part) {
    __shared__ float red[256];
    const int p = blockIdx.x * 256 + threadIdx.x;
    float L = 0.f;
    if (p < P) {
        const float *zp = z + (size_t)p * 16;
        const float *tp = target + (size_t)p * 6;
        const float invP = 1.f / (float)P;
        const float span = dh.d_max - dh.d_min;
        float dq;
        const float q = head_q(zp[0], q_ref[p], dh, dq);
        const float s = (1.f / q - dh.d_min) / span;
        const float td = (tp[0] - dh.d_min) / span;
        const float wdn = tp[5];
        const float nx = zp[1], ny = zp[2], nz = zp[3];
        const float nn = __builtin_sqrtf(nx * nx + ny * ny + nz * nz);
        const float inv = 1.f / nn;
        const float hx = nx * inv, hy = ny * inv, hz = nz * inv;
        const float cosang = hx * tp[1] + hy * tp[2] + hz * tp[3];
        const float z4 = zp[4], tc = tp[4];
        const float softplus = fmaxf(z4, 0.f) + __logf(1.f + __expf(-fabsf(z4)));
        const float diff = s - td;
        L = wdn * (fabsf(diff) + 1.f - cosang) + softplus - tc * z4;
        float g[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) g[k] = 0.f;
        const float sg = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
        g[0] = wdn * sg * (-1.f / (q * q * span)) * dq * invP;
        const float wn = -wdn * inv * invP;
        g[1] = wn * (tp[1] - cosang * hx);
        g[2] = wn * (tp[2] - cosang * hy);
        g[3] = wn * (tp[3] - cosang * hz);
        g[4] = (sigmoidf(z4) - tc) * invP;
        store8(dz + (size_t)p * 16, g);
        store8(dz + (size_t)p * 16 + 8, g + 8);
    }
    red[threadIdx.x] = L;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// sum of the per-block loss partials in a fixed order, divided by P
__global__ void loss_reduce_kernel(const float *part, int n, int P, float *loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(red[0] / (double)P);
}

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba) on the fp32 master parameters; refreshes the bf16 copy
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, bf16_t *pb, int n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float pe = p[e] - lr * (me / c1) / (__builtin_sqrtf(ve / c2) + eps);
    p[e] = pe;
    pb[e] = f2bf(pe);
}

// Training targets at the cell pixels (min(s j + s/2, W - 1), min(s i + s/2, H - 1)) of the network's grid of
// s x s cells: depth,
// normal, and the confidence C(m) = exp(-m^2 / (2 beta^2)) of Eq. 3 on the final matching cost m, twice (the
// confidence target and the weight of the depth and normal terms).
__global__ void targets_kernel(const float *depth, const float *normal, const float *cost, int W, int H, int cell,
                               int h4, int w4, float inv_2b2, float *target) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= h4 * w4) return;
    const int i = c / w4, j = c - i * w4;
    const int x = min(cell * j + cell / 2, W - 1), y = min(cell * i + cell / 2, H - 1);
    const size_t p = (size_t)y * W + x;
    const float m = cost[p];
    const float conf = expf(-m * m * inv_2b2);
    float *t = target + (size_t)c * 6;
    t[0] = depth[p];
    t[1] = normal[3 * p];
    t[2] = normal[3 * p + 1];
    t[3] = normal[3 * p + 2];
    t[4] = conf;
    t[5] = conf;
}

hipError_t launch_targets(const float *depth, const float *normal, const float *cost, int W, int H, int cell,
                          int h4, int w4, float beta, float *target, hipStream_t s) {
    const int n = h4 * w4;
    hipLaunchKernelGGL(targets_kernel, dim3((n + 255) / 256), dim3(256), 0, s, depth, normal, cost, W, H, cell, h4,
                       w4, 1.f / (2.f * beta * beta), target);
    return hipGetLastError();
}

__global__ void to_bf16_kernel(const float *src, int n, bf16_t *dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = f2bf(src[e]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline dim3 grid1(long long n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

template <int NT>
static void launch_conv_nt(const ConvArgs &a, hipStream_t s) {
    const int P = a.n * a.h * a.w;
    const dim3 grid((P + 63) / 64);
    if (a.out_f32) NN_LAUNCH((conv_kernel<NT, 1>), grid, dim3(256), 0, s, a);
    else NN_LAUNCH((conv_kernel<NT, 0>), grid, dim3(256), 0, s, a);
}

hipError_t launch_conv(const ConvArgs &a, hipStream_t s) {
    if (a.n * a.h * a.w == 0) return hipSuccess;
    switch (a.cout_pad / 16) {
        case 1: launch_conv_nt<1>(a, s); break;
        case 2: launch_conv_nt<2>(a, s); break;
        case 3: launch_conv_nt<3>(a, s); break;
        case 4: launch_conv_nt<4>(a, s); break;
        case 5: launch_conv_nt<5>(a, s); break;
        case 6: launch_conv_nt<6>(a, s); break;
        case 7: launch_conv_nt<7>(a, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs &a, float *gw, float *gb, int splits, hipStream_t s) {
    const dim3 grid(splits, (a.kpad / 16 + 3) / 4, a.cout_pad / 16);
    NN_LAUNCH(wgrad_kernel, grid, dim3(256), 0, s, a);
    const int n_w = a.cout_pad * a.kpad, n_b = a.cout_pad;
    NN_LAUNCH(wgrad_reduce_kernel, grid1(n_w + n_b), dim3(256), 0, s, a.part, a.bpart, splits, n_w, n_b, gw, gb);
    return hipGetLastError();
}

hipError_t launch_transpose_w(const bf16_t *w, int cin, int cout_pad, int kpad, int ks, bf16_t *wt, int kpad_t,
                              hipStream_t s) {
    NN_LAUNCH(transpose_w_kernel, grid1((long long)cin * kpad_t), dim3(256), 0, s, w, cin, cout_pad, kpad, ks, wt,
              kpad_t);
    return hipGetLastError();
}

hipError_t launch_pool(const bf16_t *x, int n, int h, int w, int C, bf16_t *y, hipStream_t s) {
    NN_LAUNCH(pool_kernel, grid1((long long)n * h * w * (C / 8)), dim3(256), 0, s, x, n, h, w, C, y);
    return hipGetLastError();
}

hipError_t launch_upcat(const bf16_t *low, int C1, const bf16_t *skip, int C2, int n, int h, int w, bf16_t *out,
                        hipStream_t s) {
    NN_LAUNCH(upcat_kernel, grid1((long long)n * h * w * ((C1 + C2) / 8)), dim3(256), 0, s, low, C1, skip, C2, n, h,
              w, out);
    return hipGetLastError();
}

hipError_t launch_enc_grad(const bf16_t *dp, const bf16_t *dcat, int Ccat, int off, const bf16_t *e_act, int n, int h,
                           int w, int C, bf16_t *g, hipStream_t s) {
    NN_LAUNCH(enc_grad_kernel, grid1((long long)n * h * w * (C / 8)), dim3(256), 0, s, dp, dcat, Ccat, off, e_act, n,
              h, w, C, g);
    return hipGetLastError();
}

hipError_t launch_up_grad(const bf16_t *dcat, int Ccat, const bf16_t *act, int n, int h, int w, int C1, bf16_t *g,
                          hipStream_t s) {
    NN_LAUNCH(up_grad_kernel, grid1((long long)n * h * w * (C1 / 8)), dim3(256), 0, s, dcat, Ccat, act, n, h, w, C1,
              g);
    return hipGetLastError();
}

hipError_t launch_decode(const float *z, const float *q_ref, int P, const DepthHead &dh, float *out, hipStream_t s) {
    NN_LAUNCH(decode_kernel, grid1(P), dim3(256), 0, s, z, q_ref, P, dh, out);
    return hipGetLastError();
}

int loss_blocks(int P) { return (P + 255) / 256; }

hipError_t launch_loss(const float *z, const float *q_ref, const float *target, int P, const DepthHead &dh, bf16_t *dz,
                       float *part, float *loss, hipStream_t s) {
    const int nb = loss_blocks(P);
    NN_LAUNCH(loss_kernel, dim3(nb), dim3(256), 0, s, z, q_ref, target, P, dh, dz, part);
    NN_LAUNCH(loss_reduce_kernel, dim3(1), dim3(256), 0, s, part, nb, P, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, bf16_t *pb, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
    const float c1 = 1.f - (float)std::pow((double)b1, (double)step);
    const float c2 = 1.f - (float)std::pow((double)b2, (double)step);
    NN_LAUNCH(adam_kernel, grid1(n), dim3(256), 0, s, p, g, m, v, pb, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, int n, bf16_t *dst, hipStream_t s) {
    NN_LAUNCH(to_bf16_kernel, grid1(n), dim3(256), 0, s, src, n, dst);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace amh
