// Instruction-throughput probe of the device (a measurement utility behind amh_probe_valu, not part of the
// method): the issue rate of one VALU instruction kind, from 16 independent chains per lane.  It gives the
// roofline its peak and the per-instruction costs of the evaluation's instruction mix.
#include <hip/hip_runtime.h>

#include "amhmvs.h"

namespace amh {
namespace {

constexpr int kProbeChains = 16;
constexpr int kProbeThreads = 256;

// kind: 0 v_fma_f32 (VGPR operands), 1 v_fma_f32 with an SGPR operand, 2 v_rcp_f32, 3 v_fract_f32,
// 4 v_cvt_flr_i32_f32, 5 v_med3_i32, 6 v_mad_u32_u24, 7 v_add_f32 with a literal
template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(float *out, float a, float b, int iters) {
    float x[kProbeChains];
    int n[kProbeChains];
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) {
        x[i] = 1.0f + 0.001f * (float)(threadIdx.x + i);
        n[i] = (int)threadIdx.x + i;
    }
    // the scalar arguments copied to vector registers (kind 0), so that the instruction reads no SGPR
    float av, bv;
    int lo, hi, mul;
    asm volatile("v_mov_b32 %0, %1" : "=v"(av) : "s"(a));
    asm volatile("v_mov_b32 %0, %1" : "=v"(bv) : "s"(b));
    asm volatile("v_mov_b32 %0, 0" : "=v"(lo));
    asm volatile("v_mov_b32 %0, 0x7fffffff" : "=v"(hi));
    asm volatile("v_mov_b32 %0, 3" : "=v"(mul));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kProbeChains; ++i) {
            if constexpr (KIND == 0) {
                x[i] = fmaf(x[i], av, bv);
            } else if constexpr (KIND == 1) {
                x[i] = fmaf(x[i], a, bv);
            } else if constexpr (KIND == 2) {
                x[i] = __builtin_amdgcn_rcpf(x[i]);
            } else if constexpr (KIND == 3) {
                x[i] = __builtin_amdgcn_fractf(x[i]);
            } else if constexpr (KIND == 4) {
                asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(n[i]) : "v"(x[i]));
            } else if constexpr (KIND == 5) {
                asm volatile("v_med3_i32 %0, %1, %2, %3" : "=v"(n[i]) : "v"(n[i]), "v"(lo), "v"(hi));
            } else if constexpr (KIND == 6) {
                asm volatile("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(n[i]) : "v"(n[i]), "v"(mul), "v"(lo));
            } else {
                x[i] = x[i] + 0.001f;
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) s += x[i] + (float)n[i];
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

hipError_t launch_probe(int kind, int blocks, int iters, float *out) {
    const dim3 grid((unsigned)blocks), block(kProbeThreads);
    switch (kind) {
        case 0: hipLaunchKernelGGL(probe_kernel<0>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
        case 1: hipLaunchKernelGGL(probe_kernel<1>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
        case 2: hipLaunchKernelGGL(probe_kernel<2>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
        case 3: hipLaunchKernelGGL(probe_kernel<3>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
        case 4: hipLaunchKernelGGL(probe_kernel<4>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
        case 5: hipLaunchKernelGGL(probe_kernel<5>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
        case 6: hipLaunchKernelGGL(probe_kernel<6>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
        default: hipLaunchKernelGGL(probe_kernel<7>, grid, block, 0, 0, out, 0.9999f, 0.001f, iters); break;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace amh

extern "C" amh_status amh_probe_valu(int kind, int blocks, int iters, float *ms) {
    if (kind < 0 || kind > 7 || blocks < 1 || blocks > 65536 || iters < 1 || iters > 65536 || !ms)
        return AMH_E_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AMH_E_HIP;
    float *out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * amh::kProbeThreads) != hipSuccess) return AMH_E_OOM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    amh_status st = AMH_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = AMH_E_HIP;
    if (st == AMH_OK && (amh::launch_probe(kind, 1, 1, out) != hipSuccess ||  // first launch: code load
                         hipDeviceSynchronize() != hipSuccess))
        st = AMH_E_HIP;
    if (st == AMH_OK && (hipEventRecord(e0, 0) != hipSuccess || amh::launch_probe(kind, blocks, iters, out) != hipSuccess ||
                         hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(ms, e0, e1) != hipSuccess))
        st = AMH_E_HIP;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return st;
}
