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
// Work-group: NW waves (1 or 4). A wave owns a row of 64 tile columns and RY
// tile rows; the work-group's output block is (64 t_w [x2 packed]) x
// (NW RY t_h). With NW = 1 every wave is independent (its barriers are
// wave-local), so one wave's load and sort phases overlap the networks of the
// other waves of the CU.
//   1. The union of the block's footprints is read from HBM once (coalesced,
//      replicate border by clamping) into LDS. The persistent form copies the
//      next block's union with LDS-direct loads while this block's networks
//      run.
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

// threadIdx.x as a value the compiler cannot see through: inside the
// persistent loop, addresses derived from it are recomputed per block instead
// of being hoisted out of the loop and held in registers across the networks.
__device__ __forceinline__ int mf_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Geometry of a block: the union of its tiles' footprints. The window is K
// columns by KH rows (KH = K for the square filter).
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
struct MfObGeom {
    static constexpr bool PACK = MfVTraits<V>::PACK;
    static constexpr int RX = (K - 1) / 2;         // horizontal radius
    static constexpr int RV = (KH - 1) / 2;        // vertical radius
    static constexpr int NT = 64 * NW;             // threads of a work-group
    static constexpr int TY = NW * RY;
    static constexpr int BWH = 64 * TW;            // block width of one packed half
    static constexpr int COLS = BWH + K - 1;       // footprint-union columns
    static constexpr int ROWS = TY * TH + KH - 1;  // footprint-union rows
    static constexpr int Q = (COLS + TW - 1) / TW;
    // a segment of seg_bytes starting `lead` (< 4) bytes into an aligned
    // dword needs ceil((lead + seg_bytes) / 4) <= (seg_bytes + 6) / 4 dwords;
    // they end at most 6 bytes past the segment, inside the row because of
    // the 8-element margin of the fast-path test
    static constexpr int NDMAX = (COLS * (PACK ? 2 : 4) + 6) / 4;
    static constexpr int U = (ROWS * NDMAX + NT - 1) / NT;
    // Staging buffer of the persistent form: every footprint row as whole
    // 16-byte chunks of the source row. A row needs the dwords the commit
    // reads, which end at most 18 bytes past SPAN elements from the first
    // chunk's start (see mf_obl_stage_commit).
    static constexpr int SPAN = PACK ? BWH + COLS : COLS;   // elements of a row, both halves
    static constexpr int NCH = (18 + SPAN * (PACK ? 2 : 4) + 15) / 16;   // chunks per row, widest type
    // whole 64-chunk groups: one wave instruction fills 64 consecutive chunks
    static constexpr int STG_CHUNKS = (ROWS * NCH + 63) / 64 * 64;
};

// Global loads of one block's footprint union (plain and batched forms),
// issued all at once into registers, then scattered into LDS.
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
struct MfObPrefetch {
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    uint32_t va[G::U], vb[G::PACK ? G::U : 1];
    bool fast;
};

// Blocks whose columns stay inside the image with an 8-element margin take
// the fast path: aligned dword loads of whole row segments. Blocks touching
// the left or right edge clamp element by element at commit time.
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
__device__ __forceinline__ void
mf_obl_issue(const unsigned char* __restrict__ src, int H, int W, long long pitch, int dtype, int X0, int Y0,
             MfObPrefetch<V, K, KH, TW, TH, RY, NW>& pf)
{
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    const int es = G::PACK ? (dtype == MF_U8 ? 1 : 2) : 4;
    const int gx0 = X0 - G::RX;
    const int span = G::PACK ? (G::BWH + G::COLS) : G::COLS;
    pf.fast = gx0 >= 4 && gx0 + span + 8 <= W;
    if (!pf.fast) return;
    const int nd = (G::COLS * es + 6) / 4;
    const int tid = mf_tid();
#pragma unroll
    for (int u = 0; u < G::U; ++u) {
        const int it = tid + u * G::NT;
        pf.va[u] = 0;
        if constexpr (G::PACK) pf.vb[u] = 0;
        if (it < G::ROWS * nd) {
            const int rho = it / nd, d = it - rho * nd;
            const int gy = mf_clampi(Y0 - G::RV + rho, 0, H - 1);
            const uintptr_t a = (uintptr_t)(src + (long long)gy * pitch + (long long)gx0 * es);
            const uint32_t* p = (const uint32_t*)((a & ~(uintptr_t)3) + 4 * (uintptr_t)d);
            pf.va[u] = p[0];
            if constexpr (G::PACK) pf.vb[u] = p[G::BWH * es / 4];
        }
    }
}

// Scatter the elements of one source dword into the raw buffer's row. b0 is
// the footprint column of the dword's byte 0 (may be negative); vb is the
// dword at the same position of the right half (packed types only).
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
__device__ __forceinline__ void mf_obl_put_dword(V* __restrict__ rrow, int b0, uint32_t va, uint32_t vb, int es,
                                                 int dtype)
{
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    constexpr int Q = G::Q, COLS = G::COLS;
    if constexpr (G::PACK) {
        if (es == 1) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = b0 + b;
                if (c >= 0 && c < COLS) {
                    V v;
                    v.x = (va >> (8 * b)) & 0xFF;
                    v.y = (vb >> (8 * b)) & 0xFF;
                    rrow[(c % TW) * Q + c / TW] = v;
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = (b0 >> 1) + h;  // b0 is even for 16-bit data
                if (c >= 0 && c < COLS) {
                    V v;
                    v.x = (va >> (16 * h)) & 0xFFFF;
                    v.y = (vb >> (16 * h)) & 0xFFFF;
                    rrow[(c % TW) * Q + c / TW] = v;
                }
            }
        }
    } else {
        const int c = b0 >> 2;                // 32-bit data is always aligned
        if (c >= 0 && c < COLS) {
            uint32_t b = va;
            if (dtype == MF_F32) b = mf_f32_to_key(b);
            rrow[(c % TW) * Q + c / TW] = b;
        }
    }
}

// Footprint union with clamped coordinates, element by element (blocks at
// the left or right image edge).
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
__device__ __forceinline__ void
mf_obl_load_clamped(const unsigned char* __restrict__ src, int H, int W, long long pitch, int dtype, int X0, int Y0,
                    V* __restrict__ raw)
{
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    constexpr int Q = G::Q, COLS = G::COLS;
    constexpr int UC = (G::ROWS * COLS + G::NT - 1) / G::NT;
    const int tid = mf_tid();
    // unrolled: every load of the thread is in flight at once
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        const int w = tid + u * G::NT;
        if (w >= G::ROWS * COLS) break;
        const int rho = w / COLS, c = w - rho * COLS;
        const int gy = mf_clampi(Y0 - G::RV + rho, 0, H - 1);
        const unsigned char* row = src + (long long)gy * pitch;
        const int gxa = mf_clampi(X0 - G::RX + c, 0, W - 1);
        V v;
        if constexpr (G::PACK) {
            const int gxb = mf_clampi(X0 + G::BWH - G::RX + c, 0, W - 1);
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

// Footprint union -> LDS raw buffer (swizzled layout), from the prefetched
// registers or, for edge blocks, by clamped element loads.
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
__device__ __forceinline__ void
mf_obl_commit(const unsigned char* __restrict__ src, int H, int W, long long pitch, int dtype, int X0, int Y0,
              const MfObPrefetch<V, K, KH, TW, TH, RY, NW>& pf, V* __restrict__ raw)
{
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    constexpr int Q = G::Q, COLS = G::COLS;
    const int es = G::PACK ? (dtype == MF_U8 ? 1 : 2) : 4;
    const int gx0 = X0 - G::RX;
    if (pf.fast) {
        const int nd = (COLS * es + 6) / 4;
        const int tid = mf_tid();
#pragma unroll
        for (int u = 0; u < G::U; ++u) {
            const int it = tid + u * G::NT;
            if (it < G::ROWS * nd) {
                const int rho = it / nd, d = it - rho * nd;
                const int gy = mf_clampi(Y0 - G::RV + rho, 0, H - 1);
                const uintptr_t a = (uintptr_t)(src + (long long)gy * pitch + (long long)gx0 * es);
                const int lead = (int)(a & 3);            // bytes before the segment start
                mf_obl_put_dword<V, K, KH, TW, TH, RY, NW>(raw + rho * TW * Q, 4 * d - lead, pf.va[u],
                                                       G::PACK ? pf.vb[u] : 0u, es, dtype);
            }
        }
        return;
    }
    mf_obl_load_clamped<V, K, KH, TW, TH, RY, NW>(src, H, W, pitch, dtype, X0, Y0, raw);
}

// Persistent form, stage 1a: start copying the footprint union of block
// (X0, Y0) from HBM into the LDS staging buffer with LDS-direct buffer loads
// (buffer_load_dwordx4 ... lds), which use no registers, so the copy runs
// while the networks of the current block execute. Row rho of the footprint
// lands in chunks [rho * nch, (rho + 1) * nch) as the 16-byte-aligned source
// bytes from cb, the chunk holding the row's first in-image element.
// Returns 1 for blocks whose footprint columns are all inside the image, 2
// for blocks at the left or right edge (commit clamps columns), 0 (nothing
// issued) when the caller's rows are not 16-byte aligned, or when the chunks
// would read past the end of the plane (right-edge blocks whose footprint
// reaches the last row); those blocks load element by element instead.
// Chunks may run past the end of a row into the next one (never past the
// last row's data): such bytes are never used.
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
__device__ __forceinline__ int
mf_obl_stage_issue(const unsigned char* __restrict__ src, int H, int W, long long pitch, int dtype, int X0, int Y0,
                   int aligned, uint4* stage)
{
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    const int es = G::PACK ? (dtype == MF_U8 ? 1 : 2) : 4;
    const int gx0 = X0 - G::RX;
    const int cb = (max(gx0, 0) * es) & ~15;          // first chunk, bytes from the row start
    const int nch = (18 + G::SPAN * es + 15) >> 4;
    const long long ce = cb + 16 * nch, row_bytes = (long long)W * es;
    const int gyb = mf_clampi(Y0 - G::RV, 0, H - 1);
    const int gyl = mf_clampi(Y0 - G::RV + G::ROWS - 1, 0, H - 1);
    if (!aligned || !(ce <= row_bytes || (ce <= row_bytes + pitch && gyl < H - 1))) return 0;
    // the descriptor covers the footprint's rows, up to the last chunk's end
    // (the host checks that ROWS * pitch fits in 31 bits); anything past it
    // would read as 0
    const uint32_t nrec = (uint32_t)((long long)(gyl - gyb) * pitch + max(row_bytes, ce));
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(src + (long long)gyb * pitch), (short)0, (int)nrec, 0x00020000);
    const int total = G::ROWS * nch;
    const int tid = mf_tid();
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    for (int first = wv * 64; first < total; first += G::NT) {
        const int i = first + lane;
        if (i < total) {
            const int rho = i / nch, ch = i - rho * nch;
            const int gy = mf_clampi(Y0 - G::RV + rho, 0, H - 1);
            const uint32_t off = (uint32_t)((long long)(gy - gyb) * pitch) + (uint32_t)(cb + 16 * ch);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(stage + first),
                                                     16, off, 0, 0, 0);
        }
    }
    return (gx0 >= 0 && gx0 + G::SPAN <= W) ? 1 : 2;
}

// Persistent form, stage 1b for edge blocks: staging buffer -> raw buffer
// with clamped columns. The element of global column gx sits at staging byte
// gx*es - cb of its row; for every gx the block uses,
// max(gx0, 0) <= gx <= gx0 + SPAN - 1, so it lies in [0, 16*nch).
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
__device__ __forceinline__ void mf_obl_stage_commit_clamped(const uint4* stage, int W, int dtype, int X0,
                                                            V* __restrict__ raw)
{
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    constexpr int Q = G::Q, COLS = G::COLS;
    const int es = G::PACK ? (dtype == MF_U8 ? 1 : 2) : 4;
    const int gx0 = X0 - G::RX;
    const int cb = (max(gx0, 0) * es) & ~15;
    const int nch = (18 + G::SPAN * es + 15) >> 4;
    const unsigned char* st = (const unsigned char*)stage;
    const int tid = mf_tid();
#pragma unroll 4
    for (int w = tid; w < G::ROWS * COLS; w += G::NT) {
        const int rho = w / COLS, c = w - rho * COLS;
        const unsigned char* srow = st + rho * nch * 16;
        const int gxa = mf_clampi(gx0 + c, 0, W - 1) * es - cb;
        V v;
        if constexpr (G::PACK) {
            const int gxb = mf_clampi(gx0 + G::BWH + c, 0, W - 1) * es - cb;
            if (es == 1) {
                v.x = srow[gxa];
                v.y = srow[gxb];
            } else {
                v.x = *(const uint16_t*)(srow + gxa);
                v.y = *(const uint16_t*)(srow + gxb);
            }
        } else {
            uint32_t b = *(const uint32_t*)(srow + gxa);
            if (dtype == MF_F32) b = mf_f32_to_key(b);
            v = b;
        }
        raw[(rho * TW + c % TW) * Q + c / TW] = v;
    }
}

// Persistent form, stage 1b: staging buffer -> raw buffer (swizzled, packed
// layout). Reads the same dwords as the register path: dword d of row rho
// starts at footprint column 4d - lead, at staging byte (gx0*es mod 16) rounded
// down to 4, plus 4d (+ BWH*es for the right half); the last byte read is below
// 12 + 4*nd + BWH*es <= 18 + SPAN*es, inside the row's nch chunks.
template <class V, int K, int KH, int TW, int TH, int RY, int NW>
__device__ __forceinline__ void mf_obl_stage_commit(const uint4* stage, int dtype, int X0, V* __restrict__ raw)
{
    using G = MfObGeom<V, K, KH, TW, TH, RY, NW>;
    constexpr int Q = G::Q, COLS = G::COLS;
    const int es = G::PACK ? (dtype == MF_U8 ? 1 : 2) : 4;
    const int gx0 = X0 - G::RX;
    const int nch = (18 + G::SPAN * es + 15) >> 4;
    const int a4 = ((gx0 * es) & 15) >> 2, lead = (gx0 * es) & 3;
    const int nd = (COLS * es + 6) / 4;
    const uint32_t* st = (const uint32_t*)stage;
    const int tid = mf_tid();
#pragma unroll 2
    for (int it = tid; it < G::ROWS * nd; it += G::NT) {
        const int rho = it / nd, d = it - rho * nd;
        const uint32_t* srow = st + rho * nch * 4 + a4;
        const uint32_t va = srow[d];
        const uint32_t vb = G::PACK ? srow[d + G::BWH * es / 4] : 0u;
        mf_obl_put_dword<V, K, KH, TW, TH, RY, NW>(raw + rho * TW * Q, 4 * d - lead, va, vb, es, dtype);
    }
}

// Sorted column segments of every tile row (initialisation, shared by the
// horizontally adjacent tiles of the row).
template <class NET, class V, int RY, int NW>
__device__ __forceinline__ void mf_obl_colsort(const V* __restrict__ raw, V* __restrict__ colb)
{
    using G = MfObGeom<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>;
    constexpr int TW = NET::TW, TH = NET::TH, LC = NET::LC, Q = G::Q, COLS = G::COLS;
    const int tid = mf_tid();
    // two column segments per thread in flight hide the LDS latency
#pragma unroll 2
    for (int it = tid; it < G::TY * COLS; it += G::NT) {
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
}

// Per-lane hierarchical networks of one block. With OUT_LDS = false each
// median is stored to HBM as soon as it is known; with OUT_LDS = true it goes
// to the block's LDS output tile (no bounds checks, no branches) and
// mf_obl_store_out writes the tile with 16-byte stores later.
template <class NET, class V, int RY, int NW, bool OUT_LDS = false>
__device__ __forceinline__ void
mf_obl_networks(const V* __restrict__ raw, const V* __restrict__ colb, unsigned char* __restrict__ dst, int H,
                int W, long long pitch, int dtype, int X0, int Y0, unsigned char* __restrict__ out = nullptr)
{
    using G = MfObGeom<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>;
    constexpr bool PACK = G::PACK;
    constexpr int TW = NET::TW, TH = NET::TH, LC = NET::LC, Q = G::Q, BWH = G::BWH;
    const int tid = mf_tid();
    const int lane = tid & 63, wv = tid >> 6;
    for (int ry = 0; ry < RY; ++ry) {
        const int j = wv * RY + ry;
        const V* cb = colb + j * LC * TW * Q + lane;
        const V* rb = raw + j * TH * TW * Q + lane;
        if constexpr (OUT_LDS) {
            // packed: row-major tile of 2*BWH elements of es bytes per row
            // (lanes write consecutive dwords for 8-bit data); 32-bit: planes
            // (row, px) of 64 lane-consecutive words (conflict-free)
            auto sink = [&](int px, int py, V v) {
                const int y = j * TH + py;
                if constexpr (PACK) {
                    const int xa = lane * TW + px;
                    if (dtype == MF_U8) {
                        out[y * 2 * BWH + xa] = (unsigned char)v.x;
                        out[y * 2 * BWH + xa + BWH] = (unsigned char)v.y;
                    } else {
                        ((uint16_t*)out)[y * 2 * BWH + xa] = v.x;
                        ((uint16_t*)out)[y * 2 * BWH + xa + BWH] = v.y;
                    }
                } else {
                    ((uint32_t*)out)[(y * TW + px) * 64 + lane] = (dtype == MF_F32) ? mf_key_to_f32(v) : v;
                }
            };
            NET::template run<Q>(cb, rb, sink);
        } else {
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
}

// LDS output tile of block (X0, Y0) -> HBM: 16-byte stores when the block is
// inside the image and the rows are 16-byte aligned, element stores with
// bounds checks otherwise.
template <class NET, class V, int RY, int NW>
__device__ __forceinline__ void mf_obl_store_out(const unsigned char* __restrict__ out, unsigned char* __restrict__ dst,
                                                 int H, int W, long long pitch, int dtype, int X0, int Y0,
                                                 int aligned)
{
    using G = MfObGeom<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>;
    constexpr int TW = NET::TW, BH = G::TY * NET::TH;
    constexpr int BW = G::PACK ? 2 * G::BWH : G::BWH;
    const int es = G::PACK ? (dtype == MF_U8 ? 1 : 2) : 4;
    const int cpr = BW * es / 16;                        // 16-byte chunks per tile row
    const bool whole = aligned && X0 + BW <= W;
    const int tid = mf_tid();
#pragma unroll 2
    for (int i = tid; i < BH * cpr; i += G::NT) {
        const int y = i / cpr, cx = i - y * cpr;
        if (Y0 + y >= H) break;                          // rows only grow with i
        unsigned char* row = dst + (long long)(Y0 + y) * pitch + (long long)X0 * es;
        uint32_t w[4];
        if constexpr (G::PACK) {
            const uint4 q = *(const uint4*)(out + y * BW * es + cx * 16);
            w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = 4 * cx + e;
                w[e] = ((const uint32_t*)out)[(y * TW + x % TW) * 64 + x / TW];
            }
        }
        if (whole) {
            *(uint4*)(row + cx * 16) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
            const int x0 = cx * 16 / es;                 // first element of the chunk
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int x = x0 + e / es;
                if (e % es == 0 && X0 + x < W) {
                    if (es == 1) row[x] = (unsigned char)(w[e / 4] >> (8 * (e % 4)));
                    else if (es == 2) ((uint16_t*)row)[x] = (uint16_t)(w[e / 4] >> (8 * (e % 4)));
                    else ((uint32_t*)row)[x] = w[e / 4];
                }
            }
        }
    }
}

// One work-group's block (bx, by) of one image.
template <class NET, class V, int RY, int NW>
__device__ __forceinline__ void
mf_obl_block(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
             int H, int W, long long pitch, int dtype, int bx, int by)
{
    using G = MfObGeom<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>;
    __shared__ V raw[G::ROWS * NET::TW * G::Q];
    __shared__ V colb[NET::INLINE_COLS ? 1 : G::TY * NET::LC * NET::TW * G::Q];
    const int X0 = bx * (G::PACK ? 2 * G::BWH : G::BWH);
    const int Y0 = by * (G::TY * NET::TH);
    MfObPrefetch<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW> pf;
    mf_obl_issue(src, H, W, pitch, dtype, X0, Y0, pf);
    mf_obl_commit(src, H, W, pitch, dtype, X0, Y0, pf, raw);
    __syncthreads();
    if constexpr (!NET::INLINE_COLS) {
        mf_obl_colsort<NET, V, RY, NW>(raw, colb);
        __syncthreads();
    }
    mf_obl_networks<NET, V, RY, NW>(raw, colb, dst, H, W, pitch, dtype, X0, Y0);
}

// Persistent form: work-group w filters blocks [w*per, (w+1)*per) in
// row-major order (edge blocks spread evenly over the work-groups), with no
// work-group turnover between blocks. Per block:
//   * the footprint union was copied into the LDS staging buffer by
//     LDS-direct loads issued during the previous block's networks (no
//     registers held, latency hidden); it is scattered into the raw buffer;
//   * the previous block's medians go from the LDS output tile to HBM with
//     16-byte stores, which complete during this block's networks;
//   * the next block's staging copy is issued, columns are sorted, and the
//     networks write this block's medians into the output tile.
// With TILE = false there is no output tile (less LDS, so as many
// work-groups per CU as the plain kernel): the networks store medians to HBM
// as they are produced.
template <class NET, class V, int RY, int NW, bool TILE>
__global__ void __launch_bounds__(64 * NW)
mf_obl_kernel_persistent(const unsigned char* __restrict__ src0, unsigned char* __restrict__ dst0,
                         int H, int W, long long pitch, long long plane_stride, int dtype, int nbx,
                         int nblocks, int total, int per, int aligned)
{
    using G = MfObGeom<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>;
    constexpr int BW = G::PACK ? 2 * G::BWH : G::BWH, BH = G::TY * NET::TH;
    __shared__ V raw[G::ROWS * NET::TW * G::Q];
    __shared__ V colb[NET::INLINE_COLS ? 1 : G::TY * NET::LC * NET::TW * G::Q];
    __shared__ uint4 stage[G::STG_CHUNKS];
    __shared__ uint4 out[TILE ? BH * BW * (G::PACK ? 2 : 4) / 16 : 1];
    static_assert(sizeof(raw) + sizeof(colb) + sizeof(stage) + sizeof(out) <= 160 * 1024, "LDS budget");
    // block b of the launch: plane b / nblocks, block b % nblocks of it
    const int b0 = blockIdx.x * per;
    const int b1 = min(b0 + per, total);
    if (b0 >= b1) return;
    auto plane_src = [&](int b) { return src0 + (long long)(b / nblocks) * plane_stride; };
    auto plane_dst = [&](int b) { return dst0 + (long long)(b / nblocks) * plane_stride; };
    auto bx0 = [&](int b) { return (b % nblocks % nbx) * BW; };
    auto by0 = [&](int b) { return (b % nblocks / nbx) * BH; };
    int staged = mf_obl_stage_issue<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>(
        plane_src(b0), H, W, pitch, dtype, bx0(b0), by0(b0), aligned, stage);
    for (int b = b0; b < b1; ++b) {
        const unsigned char* src = plane_src(b);
        unsigned char* dst = plane_dst(b);
        const int X0 = bx0(b), Y0 = by0(b);
        // this wave's staging copies and stores have completed; after the
        // barrier everyone's have, and the previous networks are done
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (staged == 1)
            mf_obl_stage_commit<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>(stage, dtype, X0, raw);
        else if (staged == 2)
            mf_obl_stage_commit_clamped<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>(stage, W, dtype, X0, raw);
        else
            mf_obl_load_clamped<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>(src, H, W, pitch, dtype, X0, Y0, raw);
        if (TILE && b > b0)
            mf_obl_store_out<NET, V, RY, NW>((const unsigned char*)out, plane_dst(b - 1), H, W, pitch, dtype,
                                             bx0(b - 1), by0(b - 1), aligned);
        __syncthreads();                       // raw complete; stage and out free
        staged = b + 1 >= b1 ? 0 : mf_obl_stage_issue<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>(
                                   plane_src(b + 1), H, W, pitch, dtype, bx0(b + 1), by0(b + 1), aligned, stage);
        if constexpr (!NET::INLINE_COLS) {
            mf_obl_colsort<NET, V, RY, NW>(raw, colb);
            __syncthreads();
        }
        mf_obl_networks<NET, V, RY, NW, TILE>(raw, colb, dst, H, W, pitch, dtype, X0, Y0, (unsigned char*)out);
    }
    if constexpr (TILE) {
        __syncthreads();
        mf_obl_store_out<NET, V, RY, NW>((const unsigned char*)out, plane_dst(b1 - 1), H, W, pitch, dtype,
                                         bx0(b1 - 1), by0(b1 - 1), aligned);
    }
}

template <class NET, class V, int RY, int NW>
__global__ void __launch_bounds__(64 * NW, MfVTraits<V>::PACK ? NET::MIN_WAVES : 1)
mf_obl_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
              int H, int W, long long pitch, long long plane_stride, int dtype, int nbx)
{
    const long long po = (long long)blockIdx.y * plane_stride;   // plane = blockIdx.y
    mf_obl_block<NET, V, RY, NW>(src + po, dst + po, H, W, pitch, dtype, blockIdx.x % nbx, blockIdx.x / nbx);
}

// Batched form, persistent: a resident-sized grid walks the nblocks blocks
// of every image of a job table (images sharing k, root tile and value
// class), work-group w taking blocks w, w + gridDim.x, ...; for each block it
// finds the image by binary search over the jobs' first block indices.
template <class NET, class V, int RY, int NW>
__global__ void __launch_bounds__(64 * NW, MfVTraits<V>::PACK ? NET::MIN_WAVES : 1)
mf_obl_kernel_batched(const MfJob* __restrict__ jobs, int njobs, int nblocks)
{
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].block_begin <= b) lo = mid;
            else hi = mid - 1;
        }
        const MfJob j = jobs[lo];
        const int lb = b - j.block_begin;
        mf_obl_block<NET, V, RY, NW>(j.src, j.dst, j.H, j.W, j.pitch, j.dtype, lb % j.nbx, lb / j.nbx);
        __syncthreads();   // the next block reuses the LDS
    }
}

template <class NET, class V, int RY, int NW>
static void mf_obl_batched(MfBatchedKernel* k)
{
    k->fn = (const void*)mf_obl_kernel_batched<NET, V, RY, NW>;
    k->threads = 64 * NW;
    k->lds = 0;
    k->bw = (MfVTraits<V>::PACK ? 2 : 1) * 64 * NET::TW;
    k->bh = NW * RY * NET::TH;
}

template <class NET, class V, int RY, int NW>
static hipError_t mf_obl_launch(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                                long long pitch, int dtype, hipStream_t stream)
{
    constexpr bool PACK = MfVTraits<V>::PACK;
    const int bw = (PACK ? 2 : 1) * 64 * NET::TW;
    const int bh = NW * RY * NET::TH;
    const int nbx = (W + bw - 1) / bw, nby = (H + bh - 1) / bh;
    const int nblocks = nbx * nby;
    if constexpr (NET::PERSISTENT) {
        // Persistent form, once per process from the occupancy calculator:
        // with the output tile if that fits as many work-groups per CU as the
        // plain kernel, else without it if that does; never when the kernel
        // spills to scratch. resident = 0: plain kernel only.
        static int resident = -1, tile = 0;
        if (resident < 0) {
            resident = 0;
            int per_cu_plain = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_plain, mf_obl_kernel<NET, V, RY, NW>, 64 * NW,
                                                             0) == hipSuccess && per_cu_plain >= 1) {
                const void* fns[2] = {(const void*)mf_obl_kernel_persistent<NET, V, RY, NW, true>,
                                      (const void*)mf_obl_kernel_persistent<NET, V, RY, NW, false>};
                for (int t = 0; t < 2 && resident == 0; ++t) {
                    hipFuncAttributes attr;
                    int per_cu = 0;
                    if (hipFuncGetAttributes(&attr, fns[t]) != hipSuccess || attr.localSizeBytes > 0) continue;
                    const hipError_t e = t == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                                      &per_cu, mf_obl_kernel_persistent<NET, V, RY, NW, true>,
                                                      64 * NW, 0)
                                                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                                      &per_cu, mf_obl_kernel_persistent<NET, V, RY, NW, false>,
                                                      64 * NW, 0);
                    if (e != hipSuccess || per_cu < per_cu_plain) continue;
                    if (hipGetDevice(&dev) != hipSuccess ||
                        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                        cus < 1)
                        cus = 256;
                    resident = per_cu * cus;
                    tile = t == 0;
                }
            }
        }
        const long long total = (long long)nblocks * planes;
        if (resident > 0 && total > 2LL * resident && total < (1LL << 31)) {
            const int per = (int)((total + resident - 1) / resident);
            const int grid = (int)((total + per - 1) / per);
            using G = MfObGeom<V, NET::K, NET::KH, NET::TW, NET::TH, RY, NW>;
            // LDS-direct staging and 16-byte output stores need 16-byte
            // aligned rows; buffer offsets of the footprint rows stay below 2^31
            const int aligned = ((uintptr_t)src % 16 == 0 && (uintptr_t)dst % 16 == 0 && pitch % 16 == 0 &&
                                 plane_stride % 16 == 0 && (long long)(G::ROWS + 1) * pitch < (1LL << 31)) ? 1 : 0;
            if (tile)
                hipLaunchKernelGGL((mf_obl_kernel_persistent<NET, V, RY, NW, true>), dim3(grid), dim3(64 * NW), 0,
                                   stream, (const unsigned char*)src, (unsigned char*)dst, H, W, pitch, plane_stride,
                                   dtype, nbx, nblocks, (int)total, per, aligned);
            else
                hipLaunchKernelGGL((mf_obl_kernel_persistent<NET, V, RY, NW, false>), dim3(grid), dim3(64 * NW), 0,
                                   stream, (const unsigned char*)src, (unsigned char*)dst, H, W, pitch, plane_stride,
                                   dtype, nbx, nblocks, (int)total, per, aligned);
            return hipGetLastError();
        }
    }
    // one work-group per block; grid rows are planes (at most 65535 per launch)
    for (int p0 = 0; p0 < planes; p0 += 65535) {
        const int np = planes - p0 < 65535 ? planes - p0 : 65535;
        hipLaunchKernelGGL((mf_obl_kernel<NET, V, RY, NW>), dim3(nblocks, np), dim3(64 * NW), 0, stream,
                           (const unsigned char*)src + p0 * plane_stride, (unsigned char*)dst + p0 * plane_stride,
                           H, W, pitch, plane_stride, dtype, nbx);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#define MF_OBL_INSTANTIATE(NET, RY, NW)                                                       \
    hipError_t mf_obl_launch_##NET##_r##RY##w##NW##_p16(const void* s, void* d, int np, long long ps, \
                                                        int H, int W, long long p, int dt,        \
                                                        hipStream_t st)                           \
    {                                                                                         \
        return mf_obl_launch<NET, us2, RY, NW>(s, d, np, ps, H, W, p, dt, st);                \
    }                                                                                         \
    hipError_t mf_obl_launch_##NET##_r##RY##w##NW##_u32(const void* s, void* d, int np, long long ps, \
                                                        int H, int W, long long p, int dt,        \
                                                        hipStream_t st)                           \
    {                                                                                         \
        return mf_obl_launch<NET, uint32_t, RY, NW>(s, d, np, ps, H, W, p, dt, st);           \
    }                                                                                         \
    void mf_obl_batched_##NET##_r##RY##w##NW##_p16(MfBatchedKernel* k)                       \
    {                                                                                         \
        mf_obl_batched<NET, us2, RY, NW>(k);                                                  \
    }                                                                                         \
    void mf_obl_batched_##NET##_r##RY##w##NW##_u32(MfBatchedKernel* k)                       \
    {                                                                                         \
        mf_obl_batched<NET, uint32_t, RY, NW>(k);                                             \
    }
