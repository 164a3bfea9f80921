// Calibration probe for the roofline (Sec. III): a kernel whose VALU work is
// known exactly, so that hardware counters read in one profiling run (VALU
// wave instructions, busy cycles) and the kernel's duration give the issue
// rate and clock that the rasterizers' own counters are read against.
//
// Every thread runs eight independent chains a_k <- a_k m_k + c_k of float32
// FMAs, `iters` rounds, so each wave issues exactly 8 * iters FMA
// instructions in its loop (plus a few dozen set-up and final instructions),
// with enough independent work per wave to issue back to back.
#include "rgs_internal.h"

namespace rgs {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_CHAINS = 8;

__global__ __launch_bounds__(PROBE_THREADS) void k_probe_valu(float* __restrict__ out, uint32_t iters) {
    const uint32_t gid = blockIdx.x * PROBE_THREADS + threadIdx.x;
    float a[PROBE_CHAINS], m[PROBE_CHAINS], c[PROBE_CHAINS];
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) {
        a[k] = (float)(gid & 1023u) * 1.0e-3f + (float)k;
        m[k] = 0.999f - 1.0e-4f * (float)k;
        c[k] = 1.0e-3f * (float)(k + 1);
    }
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PROBE_CHAINS; ++k) a[k] = fmaf(a[k], m[k], c[k]);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) s += a[k];
    out[gid] = s;
}

void launch_probe_valu(hipStream_t s, float* out, uint32_t blocks, uint32_t iters) {
    hipLaunchKernelGGL(k_probe_valu, dim3(blocks), dim3(PROBE_THREADS), 0, s, out, iters);
}

}  // namespace rgs
