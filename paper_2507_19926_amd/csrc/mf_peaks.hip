// Measured ceiling of the instructions the oblivious networks are made of:
// dependent chains of packed 16-bit min/max (v_pk_min_u16 / v_pk_max_u16),
// eight independent chains per lane so that issue, not latency, bounds the
// rate: kChains * 32 instructions (two 16-bit element-ops each) per lane and
// iteration.
// The bench reports the measured rate beside the public VALU peak.
#include "mf_internal.h"

namespace {

typedef unsigned short pk2 __attribute__((ext_vector_type(2)));

constexpr int kPeakThreads = 256;
constexpr int kChains = 8;

__global__ void __launch_bounds__(kPeakThreads) mf_pk_minmax_chains(uint32_t* __restrict__ out, int iters)
{
    const uint32_t t = blockIdx.x * kPeakThreads + threadIdx.x;
    pk2 x[kChains], lo, hi;
    lo.x = (unsigned short)(t * 7u);
    lo.y = (unsigned short)(t * 13u);
    hi.x = (unsigned short)(lo.x | 0x8000u);
    hi.y = (unsigned short)(lo.y | 0x8000u);
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        x[c].x = (unsigned short)(t + c * 911u);
        x[c].y = (unsigned short)(t * 3u + c);
    }
    // inline assembly: exactly kChains * 32 packed min/max per iteration,
    // whatever the compiler could prove about the values
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                asm volatile("v_pk_max_u16 %0, %0, %1" : "+v"(x[c]) : "v"(lo));
                asm volatile("v_pk_min_u16 %0, %0, %1" : "+v"(x[c]) : "v"(hi));
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= (uint32_t)x[c].x | ((uint32_t)x[c].y << 16);
    out[t] = acc;
}

}  // namespace

extern "C" int32_t mf_peak_minmax(void* out, int32_t blocks, int32_t iters, void* stream)
{
    if (!out || blocks < 1 || iters < 1) return MF_ERR_DIMS;
    hipLaunchKernelGGL(mf_pk_minmax_chains, dim3(blocks), dim3(kPeakThreads), 0, (hipStream_t)stream,
                       (uint32_t*)out, iters);
    return hipGetLastError() == hipSuccess ? MF_OK : MF_ERR_HIP;
}
