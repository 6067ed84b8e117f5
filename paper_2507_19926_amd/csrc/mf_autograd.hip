// Differentiable form of the median filter: argmedian in the forward pass and
// a deterministic gather in the backward pass. The paper has no gradients;
// the rules below are the library's.
//
// Forward: the median value comes from the hierarchical kernels; then each
// output pixel p scans its clamped k x k window in row-major order and
// records the plane-flat index of the first input pixel whose bits equal the
// median. Because clamping is monotone this is the lowest flat index among
// the window pixels holding the median.
//
// Backward: grad_in[q] = sum of grad_out[p] over output pixels p whose
// argmedian is q. Such p lie within r = (k-1)/2 of q in both directions, so
// each q gathers over its (2r+1)^2 neighbours in ascending flat order of p
// and adds in binary32 from +0. That is exactly the order of a scatter in
// ascending p, so the result is bit-reproducible and needs no atomics.
#include "mf_internal.h"

namespace {

constexpr int kBX = 64, kBY = 4;           // output block of one work-group
constexpr int kThreads = kBX * kBY;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

}  // namespace

// One work-group: a 64 x 4 block of one plane. The window union
// ((64 + k - 1) x (4 + k - 1) values) is staged in LDS as float bits.
__global__ void __launch_bounds__(kThreads)
mf_argmedian_kernel(const uint32_t* __restrict__ src, const uint32_t* __restrict__ med,
                    int32_t* __restrict__ idx, int H, int W, int k, int nbx, int nby)
{
    extern __shared__ uint32_t tile[];
    const int plane = blockIdx.x / (nbx * nby);
    const int b = blockIdx.x - plane * nbx * nby;
    const int by = b / nbx, bx = b - by * nbx;
    const int r = (k - 1) / 2;
    const long long base = (long long)plane * H * W;
    const int X0 = bx * kBX, Y0 = by * kBY;
    const int lw = kBX + 2 * r, lh = kBY + 2 * r;
    for (int i = threadIdx.x; i < lw * lh; i += kThreads) {
        const int y = i / lw, x = i - y * lw;
        const int gy = clampi(Y0 - r + y, 0, H - 1), gx = clampi(X0 - r + x, 0, W - 1);
        tile[y * lw + x] = src[base + (long long)gy * W + gx];
    }
    __syncthreads();
    const int tx = threadIdx.x % kBX, ty = threadIdx.x / kBX;
    const int y = Y0 + ty, x = X0 + tx;
    if (y >= H || x >= W) return;
    const uint32_t m = med[base + (long long)y * W + x];
    // rows in order; within a row every read is independent of the match
    // test, so the k reads of a row are in flight together
    int found = -1;
    for (int dy = 0; dy < k && found < 0; ++dy) {
        const uint32_t* row = tile + (ty + dy) * lw + tx;
        int first = k;
#pragma unroll 8
        for (int dx = 0; dx < k; ++dx)
            first = (row[dx] == m && dx < first) ? dx : first;
        if (first < k) {
            const int gy = clampi(y - r + dy, 0, H - 1), gx = clampi(x - r + first, 0, W - 1);
            found = gy * W + gx;
        }
    }
    idx[base + (long long)y * W + x] = found;
}

__global__ void __launch_bounds__(kThreads)
mf_grad_gather_kernel(const float* __restrict__ gout, const int32_t* __restrict__ idx,
                      float* __restrict__ gin, int H, int W, int k, int nbx, int nby)
{
    extern __shared__ float g[];
    const int plane = blockIdx.x / (nbx * nby);
    const int b = blockIdx.x - plane * nbx * nby;
    const int by = b / nbx, bx = b - by * nbx;
    const int r = (k - 1) / 2;
    const long long base = (long long)plane * H * W;
    const int X0 = bx * kBX, Y0 = by * kBY;
    const int lw = kBX + 2 * r, lh = kBY + 2 * r;
    int32_t* ix = reinterpret_cast<int32_t*>(g + lw * lh);
    for (int i = threadIdx.x; i < lw * lh; i += kThreads) {
        const int y = i / lw, x = i - y * lw;
        const int py = Y0 - r + y, px = X0 - r + x;
        const bool in = py >= 0 && py < H && px >= 0 && px < W;
        const long long o = base + (long long)py * W + px;
        g[i] = in ? gout[o] : 0.0f;
        ix[i] = in ? idx[o] : -1;   // -1 never equals a pixel index
    }
    __syncthreads();
    const int tx = threadIdx.x % kBX, ty = threadIdx.x / kBX;
    const int qy = Y0 + ty, qx = X0 + tx;
    if (qy >= H || qx >= W) return;
    const int q = qy * W + qx;
    float acc = 0.0f;
    // ascending p = py * W + px: rows top to bottom, columns left to right
    for (int dy = 0; dy < k; ++dy) {
        const int o = (ty + dy) * lw + tx;
        for (int dx = 0; dx < k; ++dx)
            if (ix[o + dx] == q) acc = __fadd_rn(acc, g[o + dx]);
    }
    gin[base + q] = acc;
}

hipError_t mf_ag_argmedian_launch(const float* src, const float* med, int32_t* idx, int64_t planes, int H,
                                  int W, int k, hipStream_t stream)
{
    const int nbx = (W + kBX - 1) / kBX, nby = (H + kBY - 1) / kBY;
    const long long blocks = planes * (long long)nbx * nby;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = (size_t)(kBX + k - 1) * (kBY + k - 1) * 4;
    hipLaunchKernelGGL(mf_argmedian_kernel, dim3((unsigned)blocks), dim3(kThreads), lds, stream,
                       (const uint32_t*)src, (const uint32_t*)med, idx, H, W, k, nbx, nby);
    return hipGetLastError();
}

hipError_t mf_ag_grad_launch(const float* gout, const int32_t* idx, float* gin, int64_t planes, int H, int W,
                             int k, hipStream_t stream)
{
    const int nbx = (W + kBX - 1) / kBX, nby = (H + kBY - 1) / kBY;
    const long long blocks = planes * (long long)nbx * nby;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = (size_t)(kBX + k - 1) * (kBY + k - 1) * 8;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)mf_grad_gather_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mf_grad_gather_kernel, dim3((unsigned)blocks), dim3(kThreads), lds, stream, gout,
                       idx, gin, H, W, k, nbx, nby);
    return hipGetLastError();
}
