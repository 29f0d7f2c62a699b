// Internal interface of the proposal network's kernels (amh_nn.hip).
// Activations are NHWC bf16 with channel counts that are multiples of 16;
// weights are [cout_pad][kpad] with k = tap * cin + c, tap = ky * ks + kx,
// kpad = ks^2 cin rounded up to 32, padded entries zero.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "amh_bf16.h"

namespace amh {
namespace nn {

struct ConvArgs {
    const bf16_t *x;       // [n*h*w][cin]
    const bf16_t *wgt;     // [cout_pad][kpad]
    const float *bias;     // [cout_pad] or NULL
    const bf16_t *mask;    // [n*h*w][cout_pad] or NULL: outputs where mask <= 0 are zeroed
    void *y;               // [n*h*w][cout_pad], bf16 or float
    int n, h, w;
    int cin, cout_pad, kpad, ks;
    int relu, out_f32;
};

struct WgradArgs {
    const bf16_t *x;       // [n*h*w][cin] layer input
    const bf16_t *g;       // [n*h*w][cout_pad] gradient at the layer's pre-activation
    float *part;           // [splits][cout_pad][kpad]
    float *bpart;          // [splits][cout_pad]
    int n, h, w;
    int cin, cout_pad, kpad, ks;
    int chunk;             // pixels per split (multiple of 32)
};

// depth head: depth = 1 / clamp(q_ref + R tanh(z0), q_far, q_near)
struct DepthHead {
    float d_min, d_max, q_far, q_near, R;
};

hipError_t launch_conv(const ConvArgs &a, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs &a, float *gw, float *gb, int splits, hipStream_t s);
hipError_t launch_transpose_w(const bf16_t *w, int cin, int cout_pad, int kpad, int ks, bf16_t *wt, int kpad_t,
                              hipStream_t s);
hipError_t launch_pool(const bf16_t *x, int n, int h, int w, int C, bf16_t *y, hipStream_t s);
hipError_t launch_upcat(const bf16_t *low, int C1, const bf16_t *skip, int C2, int n, int h, int w, bf16_t *out,
                        hipStream_t s);
hipError_t launch_enc_grad(const bf16_t *dp, const bf16_t *dcat, int Ccat, int off, const bf16_t *e_act, int n, int h,
                           int w, int C, bf16_t *g, hipStream_t s);
hipError_t launch_up_grad(const bf16_t *dcat, int Ccat, const bf16_t *act, int n, int h, int w, int C1, bf16_t *g,
                          hipStream_t s);
hipError_t launch_decode(const float *z, const float *q_ref, int P, const DepthHead &dh, float *out, hipStream_t s);
int loss_blocks(int P);
hipError_t launch_loss(const float *z, const float *q_ref, const float *target, int P, const DepthHead &dh, bf16_t *dz,
                       float *part, float *loss, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, bf16_t *pb, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);
hipError_t launch_to_bf16(const float *src, int n, bf16_t *dst, hipStream_t s);
hipError_t launch_targets(const float *depth, const float *normal, const float *cost, int W, int H, int cell,
                          int h4, int w4, float beta, float *target, hipStream_t s);

}  // namespace nn
}  // namespace amh
