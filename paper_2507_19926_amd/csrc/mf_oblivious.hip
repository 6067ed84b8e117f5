// Data-oblivious hierarchical-tiling median filter for gfx950 (Section 4 of
// Sugy 2025, re-designed for CDNA4).
//
// One lane owns one root tile (t_w x t_h pixels) per tile-row it visits and
// runs the generated straight-line selection network in VGPRs. For 8- and
// 16-bit data a VGPR holds two 16-bit lanes, so each lane runs two root tiles
// at once with v_pk_min_u16 / v_pk_max_u16; 32-bit data (uint32, and float32
// through an order-preserving key) uses v_min_u32 / v_max_u32 (the compiler
// fuses chains into v_min3 / v_max3).
//
// Work-group: 4 waves. A wave owns a row of 64 tile columns and RY tile rows;
// the work-group's output block is (64 t_w [x2 packed]) x (4 RY t_h).
//   1. The union of the block's footprints is read from HBM once (coalesced,
//      replicate border by clamping) into LDS.
//   2. Every footprint column segment over a tile row's core rows is sorted
//      once by one lane (odd-even merge sort in registers) and written back
//      to LDS: horizontally adjacent tiles share these sorted columns
//      (initialisation, Section 3.3).
//   3. Each lane runs the network for its tile, reading sorted columns and
//      raw corner / extra-row values from LDS at compile-time offsets, and
//      stores each median as soon as it is known.
//
// LDS layout: element (row rho, column c) of a buffer sits at
// (rho * TW + c % TW) * Q + c / TW. Lane i reads column c = i*TW + x for a
// compile-time x, so the 64 lanes of a wave touch 64 consecutive words:
// no bank conflicts in the network stage.
#pragma once

#include "mf_internal.h"

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t vmin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t vmax(uint32_t a, uint32_t b) { return a < b ? b : a; }
__device__ __forceinline__ us2 vmin(us2 a, us2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ us2 vmax(us2 a, us2 b) { return __builtin_elementwise_max(a, b); }

// float32 bit pattern <-> uint32 key whose unsigned order is IEEE totalOrder.
__device__ __forceinline__ uint32_t mf_f32_to_key(uint32_t b)
{
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ uint32_t mf_key_to_f32(uint32_t k)
{
    return k ^ ((uint32_t)((int32_t)~k >> 31) | 0x80000000u);
}

template <class V> struct MfVTraits;
template <> struct MfVTraits<us2> { static constexpr bool PACK = true; };
template <> struct MfVTraits<uint32_t> { static constexpr bool PACK = false; };

__device__ __forceinline__ int mf_clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Footprint union of one block -> LDS raw buffer (swizzled layout).
//
// Rows are clamped per row (replicate border in y). Blocks whose columns stay
// inside the image with a few bytes to spare take the fast path: every lane
// first issues all of its aligned dword loads (no dependency between them, so
// their latencies overlap), then unpacks them into LDS. Blocks touching the
// left or right edge clamp element by element.
template <class V, int K, int TW, int TH, int RY>
__device__ __forceinline__ void
mf_obl_load(const unsigned char* __restrict__ src, int H, int W, long long pitch, int dtype,
            int X0, int Y0, V* __restrict__ raw)
{
    constexpr bool PACK = MfVTraits<V>::PACK;
    constexpr int R = (K - 1) / 2;
    constexpr int TY = 4 * RY;
    constexpr int BWH = 64 * TW;
    constexpr int COLS = BWH + K - 1;
    constexpr int ROWS = TY * TH + K - 1;
    constexpr int Q = (COLS + TW - 1) / TW;
    const int es = PACK ? (dtype == MF_U8 ? 1 : 2) : 4;
    // bytes of one half-row segment, rounded out to aligned dwords
    const int seg_bytes = COLS * es;
    const int gx0 = X0 - R;                               // first column of half A
    const int span = PACK ? (BWH + COLS) : COLS;           // columns touched by the block
    const bool fast = gx0 >= 4 && gx0 + span + 8 <= W;
    if (fast) {
        // a segment of seg_bytes starting `lead` (< 4) bytes into an aligned
        // dword needs ceil((lead + seg_bytes) / 4) <= (seg_bytes + 6) / 4 dwords;
        // they end at most 6 bytes past the segment, inside the row because
        // of the 8-element margin of the fast-path test
        constexpr int NDMAX = (COLS * (PACK ? 2 : 4) + 6) / 4;
        constexpr int ITEMS = ROWS * NDMAX;
        constexpr int U = (ITEMS + 255) / 256;
        const int nd = (seg_bytes + 6) / 4;               // dwords per segment (<= NDMAX)
        uint32_t va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int it = threadIdx.x + u * 256;
            va[u] = vb[u] = 0;
            if (it < ROWS * nd) {
                const int rho = it / nd, d = it - rho * nd;
                const int gy = mf_clampi(Y0 - R + rho, 0, H - 1);
                const uintptr_t a = (uintptr_t)(src + (long long)gy * pitch + (long long)gx0 * es);
                const uint32_t* p = (const uint32_t*)((a & ~(uintptr_t)3) + 4 * (uintptr_t)d);
                va[u] = p[0];
                if constexpr (PACK) vb[u] = p[BWH * es / 4];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int it = threadIdx.x + u * 256;
            if (it < ROWS * nd) {
                const int rho = it / nd, d = it - rho * nd;
                const int gy = mf_clampi(Y0 - R + rho, 0, H - 1);
                const uintptr_t a = (uintptr_t)(src + (long long)gy * pitch + (long long)gx0 * es);
                const int lead = (int)(a & 3);            // bytes before the segment start
                const int b0 = 4 * d - lead;              // segment byte of this dword's byte 0
                V* rrow = raw + rho * TW * Q;
                if constexpr (PACK) {
                    if (es == 1) {
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int c = b0 + b;
                            if (c >= 0 && c < COLS) {
                                V v;
                                v.x = (va[u] >> (8 * b)) & 0xFF;
                                v.y = (vb[u] >> (8 * b)) & 0xFF;
                                rrow[(c % TW) * Q + c / TW] = v;
                            }
                        }
                    } else {
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int c = (b0 >> 1) + h;  // b0 is even for 16-bit data
                            if (c >= 0 && c < COLS) {
                                V v;
                                v.x = (va[u] >> (16 * h)) & 0xFFFF;
                                v.y = (vb[u] >> (16 * h)) & 0xFFFF;
                                rrow[(c % TW) * Q + c / TW] = v;
                            }
                        }
                    }
                } else {
                    const int c = b0 >> 2;                // 32-bit data is always aligned
                    if (c >= 0 && c < COLS) {
                        uint32_t b = va[u];
                        if (dtype == MF_F32) b = mf_f32_to_key(b);
                        rrow[(c % TW) * Q + c / TW] = b;
                    }
                }
            }
        }
        return;
    }
    for (int w = threadIdx.x; w < ROWS * COLS; w += 256) {
        const int rho = w / COLS, c = w - rho * COLS;
        const int gy = mf_clampi(Y0 - R + rho, 0, H - 1);
        const unsigned char* row = src + (long long)gy * pitch;
        const int gxa = mf_clampi(X0 - R + c, 0, W - 1);
        V v;
        if constexpr (PACK) {
            const int gxb = mf_clampi(X0 + BWH - R + c, 0, W - 1);
            if (dtype == MF_U8) {
                v.x = row[gxa];
                v.y = row[gxb];
            } else {
                v.x = ((const uint16_t*)row)[gxa];
                v.y = ((const uint16_t*)row)[gxb];
            }
        } else {
            uint32_t b = ((const uint32_t*)row)[gxa];
            if (dtype == MF_F32) b = mf_f32_to_key(b);
            v = b;
        }
        raw[(rho * TW + c % TW) * Q + c / TW] = v;
    }
}

// One work-group's block (bx, by) of one image.
template <class NET, class V, int RY>
__device__ __forceinline__ void
mf_obl_block(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
             int H, int W, long long pitch, int dtype, int bx, int by)
{
    constexpr bool PACK = MfVTraits<V>::PACK;
    constexpr int K = NET::K, TW = NET::TW, TH = NET::TH, LC = NET::LC;
    constexpr int R = (K - 1) / 2;
    constexpr int TX = 64;
    constexpr int TY = 4 * RY;
    constexpr int BWH = TX * TW;            // block width of one packed half
    constexpr int COLS = BWH + K - 1;       // footprint-union columns
    constexpr int ROWS = TY * TH + K - 1;   // footprint-union rows
    constexpr int Q = (COLS + TW - 1) / TW;
    __shared__ V raw[ROWS * TW * Q];
    __shared__ V colb[TY * LC * TW * Q];

    const int X0 = bx * (PACK ? 2 * BWH : BWH);
    const int Y0 = by * (TY * TH);

    // 1. footprint union -> LDS (clamped coordinates = replicate border)
    mf_obl_load<V, K, TW, TH, RY>(src, H, W, pitch, dtype, X0, Y0, raw);
    __syncthreads();

    // 2. sorted column segments over each tile row's core rows
    for (int it = threadIdx.x; it < TY * COLS; it += 256) {
        const int j = it / COLS, c = it - j * COLS;
        V a[LC];
#pragma unroll
        for (int i = 0; i < LC; ++i)
            a[i] = raw[((j * TH + TH - 1 + i) * TW + c % TW) * Q + c / TW];
        NET::sort_column(a);
#pragma unroll
        for (int i = 0; i < LC; ++i)
            colb[((j * LC + i) * TW + c % TW) * Q + c / TW] = a[i];
    }
    __syncthreads();

    // 3. per-lane hierarchical network
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int ry = 0; ry < RY; ++ry) {
        const int j = wv * RY + ry;
        const V* cb = colb + j * LC * TW * Q + lane;
        const V* rb = raw + j * TH * TW * Q + lane;
        const int ty = Y0 + j * TH, tx = X0 + lane * TW;
        auto sink = [&](int px, int py, V v) {
            const int y = ty + py;
            if (y >= H) return;
            unsigned char* row = dst + (long long)y * pitch;
            const int xa = tx + px;
            if constexpr (PACK) {
                const int xb = xa + BWH;
                if (dtype == MF_U8) {
                    if (xa < W) row[xa] = (unsigned char)v.x;
                    if (xb < W) row[xb] = (unsigned char)v.y;
                } else {
                    if (xa < W) ((uint16_t*)row)[xa] = v.x;
                    if (xb < W) ((uint16_t*)row)[xb] = v.y;
                }
            } else {
                if (xa < W) ((uint32_t*)row)[xa] = (dtype == MF_F32) ? mf_key_to_f32(v) : v;
            }
        };
        NET::template run<Q>(cb, rb, sink);
    }
}

template <class NET, class V, int RY>
__global__ void __launch_bounds__(256)
mf_obl_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
              int H, int W, long long pitch, int dtype, int nbx)
{
    mf_obl_block<NET, V, RY>(src, dst, H, W, pitch, dtype, blockIdx.x % nbx, blockIdx.x / nbx);
}

// Batched form: the grid covers the blocks of every image of a job table
// (images sharing k, root tile and value class); each work-group finds its
// image by binary search over the jobs' first block indices.
template <class NET, class V, int RY>
__global__ void __launch_bounds__(256)
mf_obl_kernel_batched(const MfJob* __restrict__ jobs, int njobs)
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
    mf_obl_block<NET, V, RY>(j.src, j.dst, j.H, j.W, j.pitch, j.dtype, lb % j.nbx, lb / j.nbx);
}

template <class NET, class V, int RY>
static void mf_obl_batched(MfBatchedKernel* k)
{
    k->fn = (const void*)mf_obl_kernel_batched<NET, V, RY>;
    k->threads = 256;
    k->lds = 0;
    k->bw = (MfVTraits<V>::PACK ? 2 : 1) * 64 * NET::TW;
    k->bh = 4 * RY * NET::TH;
}

template <class NET, class V, int RY>
static hipError_t mf_obl_launch(const void* src, void* dst, int H, int W, long long pitch,
                                int dtype, hipStream_t stream)
{
    constexpr bool PACK = MfVTraits<V>::PACK;
    const int bw = (PACK ? 2 : 1) * 64 * NET::TW;
    const int bh = 4 * RY * NET::TH;
    const int nbx = (W + bw - 1) / bw, nby = (H + bh - 1) / bh;
    hipLaunchKernelGGL((mf_obl_kernel<NET, V, RY>), dim3(nbx * nby), dim3(256), 0, stream,
                       (const unsigned char*)src, (unsigned char*)dst, H, W, pitch, dtype, nbx);
    return hipGetLastError();
}

#define MF_OBL_INSTANTIATE(NET, RY)                                                       \
    hipError_t mf_obl_launch_##NET##_p16(const void* s, void* d, int H, int W,            \
                                         long long p, int dt, hipStream_t st)            \
    {                                                                                     \
        return mf_obl_launch<NET, us2, RY>(s, d, H, W, p, dt, st);                        \
    }                                                                                     \
    hipError_t mf_obl_launch_##NET##_u32(const void* s, void* d, int H, int W,            \
                                         long long p, int dt, hipStream_t st)            \
    {                                                                                     \
        return mf_obl_launch<NET, uint32_t, RY>(s, d, H, W, p, dt, st);                   \
    }                                                                                     \
    void mf_obl_batched_##NET##_p16(MfBatchedKernel* k) { mf_obl_batched<NET, us2, RY>(k); }       \
    void mf_obl_batched_##NET##_u32(MfBatchedKernel* k) { mf_obl_batched<NET, uint32_t, RY>(k); }
