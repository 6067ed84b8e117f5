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
// The window may be rectangular (k columns by kh rows, both odd): the
// schedule encodes the recursion for its footprint, the kernel only needs the
// two radii to place the footprint.
//
// Each round is a list of merge-path chunks: a lane finds the chunk's start in
// its two sorted input windows with a co-rank binary search and then merges
// up to 16 outputs sequentially. A work-group holds T root tiles (T arenas)
// that share the schedule; a lane runs its chunk for the T tiles side by side,
// so T independent chains of LDS reads are in flight per lane. Only the ranks
// some later step can read are produced (forgetting and pruning as output
// windows).
//
// 8/16-bit data is held as 16-bit LDS elements, 32-bit data (uint32, float32
// through an order-preserving key) as 32-bit elements.
#include <mutex>

#include "mf_internal.h"
#include "mf_da_table.h"

namespace {

// one schedule: window k x kh (columns x rows), LDS element size, root tile,
// tiles per lane, lane groups per work-group
struct DaEntry {
    int k, kh, es, tw, th, tiles, groups, c_off, nchunks, r_off, nrounds, o_off, arena;
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

// G*T root tiles (bx*G*T + t, by) of one image, schedule `a`, G = a.groups.
// The work-group's lanes form G groups of kDaThreads/G lanes; group g owns
// tiles g*T .. g*T+T-1 and runs every round's chunks for them (small tiles,
// whose rounds have few chunks, fill the work-group this way). LDS holds G*T
// arenas of `arena` elements each; a lane executes each of its chunks for its
// T tiles side by side, so the T co-rank searches and loads are independent
// and their latencies overlap.
template <class E, int T>
__device__ __forceinline__ void
mf_da_block(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
            long long pitch, int dtype, const MfDaArgs& a, int bx, int by)
{
    extern __shared__ __align__(16) unsigned char mf_da_lds[];
    E* lds = reinterpret_cast<E*>(mf_da_lds);
    const int tw = a.tw, th = a.th, arena = a.arena;
    const uint32_t* __restrict__ blob = a.blob;
    const int rx = (a.k - 1) / 2, ry = (a.kh - 1) / 2;
    const int fw = a.k + tw - 1, fh = a.kh + th - 1;
    const int Y0 = by * th;
    const int G = a.groups, L = kDaThreads / G, NT = G * T;
    const int gi = threadIdx.x / L, lt = threadIdx.x - gi * L;

    // footprints -> LDS, row-major fw x fh per tile (replicate border)
    for (int i = threadIdx.x; i < NT * fw * fh; i += kDaThreads) {
        const int t = i / (fw * fh), e = i - t * fw * fh;
        const int y = e / fw, x = e - y * fw;
        const int gy = min(max(Y0 - ry + y, 0), H - 1);
        const int gx = min(max((bx * NT + t) * tw - rx + x, 0), W - 1);
        const unsigned char* row = src + (long long)gy * pitch;
        uint32_t v;
        if (dtype == MF_U8) v = row[gx];
        else if (dtype == MF_U16) v = ((const uint16_t*)row)[gx];
        else {
            v = ((const uint32_t*)row)[gx];
            if (dtype == MF_F32) v = mf_da_f32_to_key(v);
        }
        lds[t * arena + e] = (E)v;
    }
    __syncthreads();

    const uint4* __restrict__ chunks = reinterpret_cast<const uint4*>(blob + a.c_off);
    const uint32_t* __restrict__ rounds = blob + a.r_off;
    constexpr uint32_t kMask = (1u << 18) - 1;
    E* const gl = lds + gi * T * arena;     // this lane group's T arenas
    for (int rd = 0; rd < a.nrounds; ++rd) {
        const int c1 = (int)rounds[rd + 1];
        int c = (int)rounds[rd] + lt;
        uint4 d = c < c1 ? chunks[c] : make_uint4(0, 0, 0, 0);
        while (c < c1) {
            const int cn = c + L;
            const uint4 dn = cn < c1 ? chunks[cn] : make_uint4(0, 0, 0, 0);   // prefetch
            const int ao = (int)(d.x & kMask), bo = (int)(d.y & kMask), oo = (int)(d.z & kMask);
            const int na = (int)(d.x >> 18), nb = (int)(d.y >> 18), n = (int)(d.z >> 18);
            const int r0 = (int)d.w;
            // co-rank: number of A elements among the first r0 outputs (A first
            // on ties); the same bounds for every tile, so one trip count
            int lo[T], hi[T];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                lo[t] = max(0, r0 - nb);
                hi[t] = min(r0, na);
            }
            for (bool any = true; any;) {
                any = false;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    if (lo[t] < hi[t]) {
                        const E* A = gl + t * arena + ao;
                        const E* B = gl + t * arena + bo;
                        const int i = (lo[t] + hi[t]) >> 1;
                        if (A[i] <= B[r0 - i - 1]) lo[t] = i + 1;
                        else hi[t] = i;
                    }
                    any |= lo[t] < hi[t];
                }
            }
            // sequential two-pointer merge of n outputs, the T tiles side by
            // side (T independent chains of dependent LDS reads)
            if constexpr (sizeof(E) == 2) {
                // 16-bit elements in 32-bit registers: an exhausted side
                // holds 0x10000, above every element, so one compare picks
                // the side (A first on ties). pa / pb are the arena indices
                // of the heads, ea / eb one past the windows.
                constexpr uint32_t kDone = 0x10000u;
                int pa[T], pb[T];
                uint32_t va[T], vb[T];
                const int ea = ao + na, eb = bo + nb;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    pa[t] = ao + lo[t];
                    pb[t] = bo + r0 - lo[t];
                    va[t] = pa[t] < ea ? (uint32_t)gl[t * arena + pa[t]] : kDone;
                    vb[t] = pb[t] < eb ? (uint32_t)gl[t * arena + pb[t]] : kDone;
                }
                for (int q = 0; q < n; ++q) {
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        const bool takeA = va[t] <= vb[t];
                        gl[t * arena + oo + q] = (E)min(va[t], vb[t]);
                        pa[t] += takeA ? 1 : 0;
                        pb[t] += takeA ? 0 : 1;
                        const int p = takeA ? pa[t] : pb[t];
                        const int e = takeA ? ea : eb;
                        // index clamped into the arena; past the window the
                        // value is replaced by kDone
                        const uint32_t nv = (uint32_t)gl[t * arena + min(p, arena - 1)];
                        const uint32_t nk = p < e ? nv : kDone;
                        va[t] = takeA ? nk : va[t];
                        vb[t] = takeA ? vb[t] : nk;
                    }
                }
            } else {
                int ii[T], jj[T];
                E va[T], vb[T];
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const E* A = gl + t * arena + ao;
                    const E* B = gl + t * arena + bo;
                    ii[t] = lo[t];
                    jj[t] = r0 - lo[t];
                    va[t] = ii[t] < na ? A[ii[t]] : (E)0;
                    vb[t] = jj[t] < nb ? B[jj[t]] : (E)0;
                }
                for (int q = 0; q < n; ++q) {
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        const bool takeA = (ii[t] < na) && (jj[t] >= nb || va[t] <= vb[t]);
                        gl[t * arena + oo + q] = takeA ? va[t] : vb[t];
                        ii[t] += takeA ? 1 : 0;
                        jj[t] += takeA ? 0 : 1;
                        // one read refills the side just consumed; the index is
                        // clamped into the arena (an exhausted side is never used)
                        const int src_i = takeA ? ao + ii[t] : bo + jj[t];
                        const E nv = gl[t * arena + min(src_i, arena - 1)];
                        va[t] = takeA ? nv : va[t];
                        vb[t] = takeA ? vb[t] : nv;
                    }
                }
            }
            d = dn;
            c = cn;
        }
        __syncthreads();
    }

    const uint32_t* outs = blob + a.o_off;
    for (int p = threadIdx.x; p < NT * tw * th; p += kDaThreads) {
        const int t = p / (tw * th), e = p - t * tw * th;
        const int y = Y0 + e / tw, x = (bx * NT + t) * tw + e % tw;
        if (y >= H || x >= W) continue;
        unsigned char* row = dst + (long long)y * pitch;
        const uint32_t v = (uint32_t)lds[t * arena + outs[e]];
        if (dtype == MF_U8) row[x] = (unsigned char)v;
        else if (dtype == MF_U16) ((uint16_t*)row)[x] = (uint16_t)v;
        else ((uint32_t*)row)[x] = (dtype == MF_F32) ? mf_da_key_to_f32(v) : v;
    }
}

template <class E, int T>
__global__ void __launch_bounds__(kDaThreads)
mf_da_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
             long long pitch, long long plane_stride, int dtype, MfDaArgs a, int ntx)
{
    const long long po = (long long)blockIdx.y * plane_stride;   // plane = blockIdx.y
    mf_da_block<E, T>(src + po, dst + po, H, W, pitch, dtype, a, blockIdx.x % ntx, blockIdx.x / ntx);
}

// Batched form: blocks of every image of a job table (same k, tile, tiles per
// work-group and element size), image found by binary search over first
// block indices.
template <class E, int T>
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
    mf_da_block<E, T>(j.src, j.dst, j.H, j.W, j.pitch, j.dtype, a, lb % j.nbx, lb / j.nbx);
}

namespace {

// kernel pointers by (element size, tiles per work-group)
template <class E>
const void* da_kernel(int T, bool batched)
{
    switch (T) {
    case 1: return batched ? (const void*)mf_da_kernel_batched<E, 1> : (const void*)mf_da_kernel<E, 1>;
    case 2: return batched ? (const void*)mf_da_kernel_batched<E, 2> : (const void*)mf_da_kernel<E, 2>;
    default: return batched ? (const void*)mf_da_kernel_batched<E, 4> : (const void*)mf_da_kernel<E, 4>;
    }
}

const void* da_kernel_for(const DaEntry* e, bool batched)
{
    return e->es == 2 ? da_kernel<uint16_t>(e->tiles, batched) : da_kernel<uint32_t>(e->tiles, batched);
}

}  // namespace

namespace {

// kh = 0: the square k x k window
const DaEntry* da_find(int dtype, int k, int tw, int th, int group, int kh = 0)
{
    const int es = (dtype == MF_U8 || dtype == MF_U16) ? 2 : 4;
    if (kh == 0) kh = k;
    for (int i = 0; i < kDaCount; ++i) {
        const DaEntry& e = kDaTable[i];
        if (e.k == k && e.kh == kh && e.es == es && (tw == 0 || e.tw == tw) && (th == 0 || e.th == th) &&
            (group == 0 || e.tiles == group))
            return &e;
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
        for (int es = 2; es <= 4; es += 2)
            for (int T = 1; T <= 4; T *= 2)
                for (int bt = 0; bt < 2; ++bt) {
                    const void* fn = es == 2 ? da_kernel<uint16_t>(T, bt) : da_kernel<uint32_t>(T, bt);
                    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
                    if (e != hipSuccess) return e;
                }
        g_da_blob_dev[dev] = (const uint32_t*)p;
    }
    *out = g_da_blob_dev[dev];
    return hipSuccess;
}

}  // namespace

bool mf_da_supports(int dtype, int k, int tw, int th, int group, int kh)
{
    return da_find(dtype, k, tw, th, group, kh) != nullptr;
}

int mf_da_rect_max_side() { return MF_DA_RECT_MAX_SIDE; }

void mf_da_default_tile(int dtype, int k, int* tw, int* th, int* group, int kh)
{
    const DaEntry* e = da_find(dtype, k, 0, 0, 0, kh);
    *tw = e ? e->tw : 0;
    *th = e ? e->th : 0;
    *group = e ? e->tiles : 0;
}

int mf_da_list(int dtype, int k, int* tw, int* th, int* group, int cap)
{
    const int es = (dtype == MF_U8 || dtype == MF_U16) ? 2 : 4;
    int n = 0;
    for (int i = 0; i < kDaCount; ++i) {
        const DaEntry& e = kDaTable[i];
        if (e.k != k || e.kh != k || e.es != es) continue;
        if (n < cap) {
            tw[n] = e.tw;
            th[n] = e.th;
            group[n] = e.tiles;
        }
        ++n;
    }
    return n;
}

static MfDaArgs da_args(const DaEntry* e, const uint32_t* blob)
{
    MfDaArgs a;
    a.blob = blob;
    a.k = e->k;
    a.kh = e->kh;
    a.tw = e->tw;
    a.th = e->th;
    a.c_off = e->c_off;
    a.r_off = e->r_off;
    a.nrounds = e->nrounds;
    a.o_off = e->o_off;
    a.arena = e->arena;
    a.groups = e->groups;
    return a;
}

hipError_t mf_da_launch(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                        long long pitch, int dtype, int k, int tw, int th, int group, hipStream_t stream, int kh)
{
    const DaEntry* e = da_find(dtype, k, tw, th, group, kh);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    MfDaArgs a = da_args(e, blob);
    const int bw = e->tw * e->tiles * e->groups;     // pixels of a work-group along x
    const int ntx = (W + bw - 1) / bw, nty = (H + e->th - 1) / e->th;
    if ((long long)ntx * nty > 0x7fffffffLL) return hipErrorInvalidConfiguration;   // grid.x limit
    const size_t lds = (size_t)e->arena * e->es * e->tiles * e->groups;
    for (int p0 = 0; p0 < planes; p0 += 65535) {     // grid rows are planes
        const int np = planes - p0 < 65535 ? planes - p0 : 65535;
        const unsigned char* s8 = (const unsigned char*)src + p0 * plane_stride;
        unsigned char* d8 = (unsigned char*)dst + p0 * plane_stride;
        void* args[] = {&s8, &d8, &H, &W, &pitch, &plane_stride, &dtype, &a, (void*)&ntx};
        err = hipLaunchKernel(da_kernel_for(e, false), dim3(ntx * nty, np), dim3(kDaThreads), args, lds, stream);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t mf_da_batched(int dtype, int k, int tw, int th, int group, MfBatchedKernel* kern, MfDaArgs* args)
{
    const DaEntry* e = da_find(dtype, k, tw, th, group);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    *args = da_args(e, blob);
    kern->fn = da_kernel_for(e, true);
    kern->threads = kDaThreads;
    kern->lds = (size_t)e->arena * e->es * e->tiles * e->groups;
    kern->bw = e->tw * e->tiles * e->groups;
    kern->bh = e->th;
    return hipSuccess;
}
