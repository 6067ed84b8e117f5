// Data-aware hierarchical-tiling median filter for gfx950 (Section 5 of
// Sugy 2025, re-designed around LDS residency).
//
// One work-group owns one root tile. Its footprint is read from HBM into LDS
// once; then a precomputed schedule of two-way merges runs entirely in LDS:
// column sorts, extra-row sorts and corner sorts as binary reductions from
// single values, the core's multi-way merge as a binary reduction of sorted
// columns, and every split's core and row/column extensions level by level
// (Sections 3.3-3.4, 5.1). The paper's global-memory multi-pass structure is
// replaced by this LDS-resident sequence of rounds separated by barriers.
//
// Each round is a list of merge-path chunks: a lane finds the chunk's start in
// its two sorted input windows with a co-rank binary search and then merges
// up to 16 outputs sequentially. Only the ranks some later step can read are
// produced (forgetting and pruning as output windows).
//
// 8/16-bit data is held as 16-bit LDS elements, 32-bit data (uint32, float32
// through an order-preserving key) as 32-bit elements.
#include <mutex>

#include "mf_internal.h"
#include "mf_da_table.h"

namespace {

struct DaEntry {
    int k, es, tw, th, c_off, nchunks, r_off, nrounds, o_off, arena;
};

const DaEntry kDaTable[] = {MF_DA_TABLE_ENTRIES};
constexpr int kDaCount = sizeof(kDaTable) / sizeof(kDaTable[0]);

constexpr int kDaThreads = 512;

}  // namespace

extern "C" const unsigned char mf_da_blob_host[];

// All schedules; copied from the host image once per device.
__device__ __align__(16) uint32_t mf_da_blob[MF_DA_BLOB_WORDS];

__device__ __forceinline__ uint32_t mf_da_f32_to_key(uint32_t b)
{
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ uint32_t mf_da_key_to_f32(uint32_t k)
{
    return k ^ ((uint32_t)((int32_t)~k >> 31) | 0x80000000u);
}

// Root tile (bx, by) of one image, schedule `a`.
template <class E>
__device__ __forceinline__ void
mf_da_block(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
            long long pitch, int dtype, const MfDaArgs& a, int bx, int by)
{
    extern __shared__ __align__(16) unsigned char mf_da_lds[];
    E* lds = reinterpret_cast<E*>(mf_da_lds);
    const int k = a.k, tw = a.tw, th = a.th;
    const uint32_t* __restrict__ blob = a.blob;
    const int c_off = a.c_off, r_off = a.r_off, nrounds = a.nrounds, o_off = a.o_off;
    const int X0 = bx * tw, Y0 = by * th;
    const int r = (k - 1) / 2;
    const int fw = k + tw - 1, fh = k + th - 1;

    // footprint -> LDS, row-major fw x fh (replicate border by clamping)
    for (int i = threadIdx.x; i < fw * fh; i += kDaThreads) {
        const int y = i / fw, x = i - y * fw;
        const int gy = min(max(Y0 - r + y, 0), H - 1);
        const int gx = min(max(X0 - r + x, 0), W - 1);
        const unsigned char* row = src + (long long)gy * pitch;
        uint32_t v;
        if (dtype == MF_U8) v = row[gx];
        else if (dtype == MF_U16) v = ((const uint16_t*)row)[gx];
        else {
            v = ((const uint32_t*)row)[gx];
            if (dtype == MF_F32) v = mf_da_f32_to_key(v);
        }
        lds[i] = (E)v;
    }
    __syncthreads();

    const uint4* chunks = reinterpret_cast<const uint4*>(blob + c_off);
    const uint32_t* rounds = blob + r_off;
    constexpr uint32_t kMask = (1u << 18) - 1;
    for (int rd = 0; rd < nrounds; ++rd) {
        const int c1 = (int)rounds[rd + 1];
        for (int c = (int)rounds[rd] + threadIdx.x; c < c1; c += kDaThreads) {
            const uint4 d = chunks[c];
            const E* A = lds + (d.x & kMask);
            const E* B = lds + (d.y & kMask);
            E* O = lds + (d.z & kMask);
            const int na = (int)(d.x >> 18), nb = (int)(d.y >> 18), n = (int)(d.z >> 18);
            const int r0 = (int)d.w;
            // co-rank: number of A elements among the first r0 merged outputs
            // (A first on ties)
            int lo = max(0, r0 - nb), hi = min(r0, na);
            while (lo < hi) {
                const int i = (lo + hi) >> 1;
                if (A[i] <= B[r0 - i - 1]) lo = i + 1;
                else hi = i;
            }
            int i = lo, j = r0 - lo;
            E a = 0, b = 0;
            if (i < na) a = A[i];
            if (j < nb) b = B[j];
            for (int t = 0; t < n; ++t) {
                const bool takeA = (i < na) && (j >= nb || a <= b);
                O[t] = takeA ? a : b;
                if (takeA) {
                    ++i;
                    if (i < na) a = A[i];
                } else {
                    ++j;
                    if (j < nb) b = B[j];
                }
            }
        }
        __syncthreads();
    }

    const uint32_t* outs = blob + o_off;
    for (int p = threadIdx.x; p < tw * th; p += kDaThreads) {
        const int y = Y0 + p / tw, x = X0 + p % tw;
        if (y >= H || x >= W) continue;
        unsigned char* row = dst + (long long)y * pitch;
        const uint32_t v = (uint32_t)lds[outs[p]];
        if (dtype == MF_U8) row[x] = (unsigned char)v;
        else if (dtype == MF_U16) ((uint16_t*)row)[x] = (uint16_t)v;
        else ((uint32_t*)row)[x] = (dtype == MF_F32) ? mf_da_key_to_f32(v) : v;
    }
}

template <class E>
__global__ void __launch_bounds__(kDaThreads)
mf_da_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
             long long pitch, int dtype, MfDaArgs a, int ntx)
{
    mf_da_block<E>(src, dst, H, W, pitch, dtype, a, blockIdx.x % ntx, blockIdx.x / ntx);
}

// Batched form: blocks of every image of a job table (same k, tile and
// element size), image found by binary search over first block indices.
template <class E>
__global__ void __launch_bounds__(kDaThreads)
mf_da_kernel_batched(const MfJob* __restrict__ jobs, int njobs, MfDaArgs a)
{
    const int b = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const MfJob j = jobs[lo];
    const int lb = b - j.block_begin;
    mf_da_block<E>(j.src, j.dst, j.H, j.W, j.pitch, j.dtype, a, lb % j.nbx, lb / j.nbx);
}

namespace {

const DaEntry* da_find(int dtype, int k, int tw, int th)
{
    const int es = (dtype == MF_U8 || dtype == MF_U16) ? 2 : 4;
    for (int i = 0; i < kDaCount; ++i) {
        const DaEntry& e = kDaTable[i];
        if (e.k == k && e.es == es && (tw == 0 || e.tw == tw) && (th == 0 || e.th == th)) return &e;
    }
    return nullptr;
}

std::mutex g_da_mu;
const uint32_t* g_da_blob_dev[64];

// Device copy of the schedules for the current device (copied once).
hipError_t da_blob(const uint32_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_da_mu);
    if (!g_da_blob_dev[dev]) {
        e = hipMemcpyToSymbol(HIP_SYMBOL(mf_da_blob), mf_da_blob_host, sizeof(uint32_t) * MF_DA_BLOB_WORDS, 0,
                              hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(mf_da_blob));
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)mf_da_kernel<uint16_t>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)mf_da_kernel<uint32_t>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)mf_da_kernel_batched<uint16_t>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)mf_da_kernel_batched<uint32_t>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        g_da_blob_dev[dev] = (const uint32_t*)p;
    }
    *out = g_da_blob_dev[dev];
    return hipSuccess;
}

}  // namespace

bool mf_da_supports(int dtype, int k, int tw, int th) { return da_find(dtype, k, tw, th) != nullptr; }

void mf_da_default_tile(int dtype, int k, int* tw, int* th)
{
    const DaEntry* e = da_find(dtype, k, 0, 0);
    *tw = e ? e->tw : 0;
    *th = e ? e->th : 0;
}

static MfDaArgs da_args(const DaEntry* e, const uint32_t* blob)
{
    MfDaArgs a;
    a.blob = blob;
    a.k = e->k;
    a.tw = e->tw;
    a.th = e->th;
    a.c_off = e->c_off;
    a.r_off = e->r_off;
    a.nrounds = e->nrounds;
    a.o_off = e->o_off;
    return a;
}

hipError_t mf_da_launch(const void* src, void* dst, int H, int W, long long pitch, int dtype, int k,
                        int tw, int th, hipStream_t stream)
{
    const DaEntry* e = da_find(dtype, k, tw, th);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    const MfDaArgs a = da_args(e, blob);
    const int ntx = (W + e->tw - 1) / e->tw, nty = (H + e->th - 1) / e->th;
    const size_t lds = (size_t)e->arena * e->es;
    if (e->es == 2)
        hipLaunchKernelGGL(mf_da_kernel<uint16_t>, dim3(ntx * nty), dim3(kDaThreads), lds, stream,
                           (const unsigned char*)src, (unsigned char*)dst, H, W, pitch, dtype, a, ntx);
    else
        hipLaunchKernelGGL(mf_da_kernel<uint32_t>, dim3(ntx * nty), dim3(kDaThreads), lds, stream,
                           (const unsigned char*)src, (unsigned char*)dst, H, W, pitch, dtype, a, ntx);
    return hipGetLastError();
}

hipError_t mf_da_batched(int dtype, int k, int tw, int th, MfBatchedKernel* kern, MfDaArgs* args)
{
    const DaEntry* e = da_find(dtype, k, tw, th);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    *args = da_args(e, blob);
    kern->fn = e->es == 2 ? (const void*)mf_da_kernel_batched<uint16_t> : (const void*)mf_da_kernel_batched<uint32_t>;
    kern->threads = kDaThreads;
    kern->lds = (size_t)e->arena * e->es;
    kern->bw = e->tw;
    kern->bh = e->th;
    return hipSuccess;
}
