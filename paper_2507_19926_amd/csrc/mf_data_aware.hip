// Data-aware hierarchical-tiling median filter for gfx950 (Section 5 of
// Sugy 2025, re-designed around LDS residency).
//
// One work-group owns one root tile (or G small ones, one per lane group).
// Its footprint is read from HBM into LDS once; then a precomputed schedule
// runs entirely in LDS, round after round with a work-group barrier between
// rounds: column, extra-row and corner sorts as per-lane sorting networks
// over footprint values in registers (Section 5.1), the core's multi-way
// merge as a binary reduction of two-way merges of sorted columns, and every
// split's core and row/column extensions level by level (Sections 3.3-3.4).
// The paper's global-memory multi-pass structure is replaced by this
// LDS-resident sequence of rounds.
//
// The window may be rectangular (k columns by kh rows, both odd): the
// schedule encodes the recursion for its footprint, the kernel only needs the
// two radii to place the footprint.
//
// A merge is cut into chunks of one length per round: a lane finds its
// chunk's start in the two sorted input windows with a co-rank binary search
// (run as a wave-uniform loop of the wave's largest step count) and then
// emits four outputs per step: the four smallest of the next four elements
// of each input, by a half-cleaner and a bitonic sort of four (every stored
// list ends with sentinels, so no step tests for an exhausted input). Only
// the ranks some later step can read are produced (forgetting and pruning as
// output windows).
//
// 8-bit data is held as 8-bit LDS elements (16-bit in the global-memory
// form), 16-bit data as 16-bit elements, 32-bit data (uint32, float32 through
// an order-preserving key) as 32-bit elements; 8- and 16-bit steps work on
// packed 16-bit pairs. Steps and sort items address the LDS arena by byte
// address; when a lane group spans whole waves the arena base (and, for 8-
// and 16-bit elements, the item loop) lives in scalar registers. Work-groups
// of the one-plane and 3-D kernels take their tiles in contiguous runs per
// XCD, so each L2 serves neighbouring footprints.
#include <mutex>

#include "mf_internal.h"
#include "mf_da_table.h"

namespace {

// one schedule: window k x kh (columns x rows; k x kh x kz for a 3-D box,
// kz = 1 for planes), element size, root tile tw x th (x tz), tiles per lane
// (always 1), lane groups per work-group, memory (0: LDS
// arena, 1: device workspace of the global form), round mode (0: rounds per
// recursion level, 1: rounds over the whole schedule), blob offsets of the items,
// round boundaries, per-round chunk lengths, per-round recursion levels and
// median offsets, arena elements
struct DaEntry {
    int k, kh, kz, es, tw, th, tz, tiles, groups, mem, mode, c_off, nchunks, r_off, nrounds, l_off, p_off, o_off,
        arena;
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

// Arena addressing of the sort items and the 8- and 16-bit merge steps.
// With the arena in LDS (LDS = true) a location is its LDS byte address: no
// base register to add per access. The global-memory form keeps the arena in
// device memory; there a location is a byte offset from the arena base gb.
typedef __attribute__((address_space(3))) uint32_t mf_lds_u32;
typedef uint32_t mf_u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t mf_u32x4 __attribute__((ext_vector_type(4)));
template <bool LDS>
__device__ __forceinline__ uint32_t mf_da_addr(const unsigned char* gb, const void* p)
{
    if constexpr (LDS)
        return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) unsigned char*)p;
    else
        return (uint32_t)((const unsigned char*)p - gb);
}
// the aligned dword holding location x
template <bool LDS>
__device__ __forceinline__ auto mf_da_dw(const unsigned char* gb, uint32_t x)
{
    if constexpr (LDS)
        return (const mf_lds_u32*)(uintptr_t)(x & ~3u);
    else
        return reinterpret_cast<const uint32_t*>(gb + (x & ~3u));
}
template <bool LDS, class T>
__device__ __forceinline__ void mf_da_put(unsigned char* gb, uint32_t x, T v)
{
    if constexpr (LDS)
        *(__attribute__((address_space(3))) T*)(uintptr_t)x = v;
    else
        *reinterpret_cast<T*>(gb + x) = v;
}
template <bool LDS, class E>
__device__ __forceinline__ E mf_da_get(const unsigned char* gb, uint32_t x)
{
    if constexpr (LDS)
        return *(const __attribute__((address_space(3))) E*)(uintptr_t)x;
    else
        return *reinterpret_cast<const E*>(gb + x);
}

// Batcher's odd-even merge sort of N (a power of two) values in registers,
// fully unrolled: every index is a compile-time constant.
template <int N>
__device__ __forceinline__ void mf_da_sortnet(uint32_t* v)
{
#pragma unroll
    for (int p = 1; p < N; p <<= 1)
#pragma unroll
        for (int k = p; k >= 1; k >>= 1)
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
                for (int i = 0; i < k; ++i)
                    if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        const uint32_t x = v[i + j], y = v[i + j + k];
                        v[i + j] = min(x, y);
                        v[i + j + k] = max(x, y);
                    }
}

// Sort item: the n*L footprint values at base + j*lstep + i*stride (L
// parallel lines of n values; padded to N with the sentinel), sorted by the
// network; ranks [lo, lo+cnt) are written from out, followed by MF_DA_SENT
// sentinels.
template <class E, int N, bool LDS>
__device__ __forceinline__ void mf_da_sort(E* __restrict__ gl, const uint4 d)
{
    constexpr uint32_t kMask = (1u << 18) - 1;
    constexpr uint32_t kMax = (uint32_t)(E)~(E)0;
    constexpr uint32_t es = sizeof(E);
    const int base = (int)(d.x & kMask), n = (int)(d.x >> 18);
    const int stride = (int)(d.y & kMask), lo = (int)(d.y >> 18);
    const int oo = (int)(d.z & kMask), cnt = (int)(d.z >> 18);
    const int lines = (int)((d.w >> 6) & 7u), lstep = (int)((d.w >> 9) & ((1u << 22) - 1));
    const int total = n * lines;
    // locations as in the merge steps (LDS byte addresses in LDS arenas), so
    // that the arena base is needed once per item, not per value
    unsigned char* gb = reinterpret_cast<unsigned char*>(gl);
    const uint32_t xs = (uint32_t)stride * es, xback = ((uint32_t)lstep - (uint32_t)(n * stride)) * es;
    uint32_t v[N];
    int e = 0;
    uint32_t x = mf_da_addr<LDS>(gb, gl + base);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        v[i] = i < total ? (uint32_t)mf_da_get<LDS, E>(gb, x) : kMax;
        // next value: along the line, or the first of the next line
        ++e;
        x += xs;
        const bool wrap = e == n;
        e = wrap ? 0 : e;
        x = wrap ? x + xback : x;
    }
    mf_da_sortnet<N>(v);
    const uint32_t xo = mf_da_addr<LDS>(gb, gl + oo) - (uint32_t)lo * es;
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i >= lo && i < lo + cnt) mf_da_put<LDS>(gb, xo + (uint32_t)i * es, (E)v[i]);
    const uint32_t xe = mf_da_addr<LDS>(gb, gl + oo + cnt);
#pragma unroll
    for (int i = 0; i < MF_DA_SENT; ++i) mf_da_put<LDS>(gb, xe + (uint32_t)i * es, (E)kMax);
}

// Two 16-bit values per 32-bit register (element 2j in the low half).
typedef unsigned short mf_u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t mf_pk_min(uint32_t x, uint32_t y)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(mf_u16x2, x),
                                                                  __builtin_bit_cast(mf_u16x2, y)));
}
__device__ __forceinline__ uint32_t mf_pk_max(uint32_t x, uint32_t y)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(mf_u16x2, x),
                                                                  __builtin_bit_cast(mf_u16x2, y)));
}
// Per half, 1 where x > y, else 0: min(max(x - y, 0), 1) on both halves at
// once. Written as the two instructions themselves: the compiler otherwise
// turns the expression into per-half compares and selects.
__device__ __forceinline__ uint32_t mf_pk_gt01(uint32_t x, uint32_t y)
{
    uint32_t d, r;
    asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(d) : "v"(x), "v"(y));
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(d), "s"(0x00010001u));
    return r;
}
__device__ __forceinline__ uint32_t mf_swap16(uint32_t x) { return __builtin_amdgcn_alignbit(x, x, 16); }

// [a0 <= b0] + [a1 <= b1] + [a2 <= b2] + [a3 <= b3] (unsigned): a compare
// per pair, the first result selected as 0/1, the others added through the
// carry. Written as the instructions themselves: the compiler otherwise builds
// a bit mask and counts its bits, twice the instructions.
__device__ __forceinline__ uint32_t mf_count_le4(uint32_t a0, uint32_t b0, uint32_t a1, uint32_t b1, uint32_t a2,
                                                 uint32_t b2, uint32_t a3, uint32_t b3)
{
    uint32_t n;
    asm("v_cmp_le_u32 vcc, %1, %2\n\t"
        "v_cndmask_b32 %0, 0, 1, vcc\n\t"
        "v_cmp_le_u32 vcc, %3, %4\n\t"
        "v_addc_co_u32 %0, vcc, 0, %0, vcc\n\t"
        "v_cmp_le_u32 vcc, %5, %6\n\t"
        "v_addc_co_u32 %0, vcc, 0, %0, vcc\n\t"
        "v_cmp_le_u32 vcc, %7, %8\n\t"
        "v_addc_co_u32 %0, vcc, 0, %0, vcc"
        : "=&v"(n)
        : "v"(a0), "v"(b0), "v"(a1), "v"(b1), "v"(a2), "v"(b2), "v"(a3), "v"(b3)
        : "vcc");
    return n;
}

// Bytes of v spread by selector sel into the 16-bit halves (v_perm with a
// zero first source). The selector is taken from a scalar register: as a
// constant the compiler keeps it in a vector register, which in the 64-VGPR
// builds it rematerialises at every step.
__device__ __forceinline__ uint32_t mf_perm0(uint32_t v, uint32_t sel)
{
    uint32_t r;
    asm("v_perm_b32 %0, 0, %1, %2" : "=v"(r) : "v"(v), "s"(sel));
    return r;
}

// Four consecutive 8-bit elements from location x on, widened to the 16-bit
// pairs (x, x+1) and (x+2, x+3): the two aligned dwords that hold them,
// shifted into place (v_alignbyte takes the shift from the location's low
// two bits), then spread over 16-bit halves. _rev gives the four in reverse
// order, as the pairs (x+3, x+2) and (x+1, x).
template <bool LDS>
__device__ __forceinline__ uint32_t mf_da_at4_u8(const unsigned char* gb, uint32_t x)
{
    const auto w = mf_da_dw<LDS>(gb, x);
    return __builtin_amdgcn_alignbyte(w[1], w[0], x);
}
template <bool LDS>
__device__ __forceinline__ void mf_da_get4_u8(const unsigned char* gb, uint32_t x, uint32_t& lo, uint32_t& hi)
{
    const uint32_t v = mf_da_at4_u8<LDS>(gb, x);
    lo = mf_perm0(v, 0x0c010c00u);
    hi = mf_perm0(v, 0x0c030c02u);
}
template <bool LDS>
__device__ __forceinline__ void mf_da_get4_u8_rev(const unsigned char* gb, uint32_t x, uint32_t& r32,
                                                  uint32_t& r10)
{
    const uint32_t v = mf_da_at4_u8<LDS>(gb, x);
    r32 = mf_perm0(v, 0x0c020c03u);
    r10 = mf_perm0(v, 0x0c000c01u);
}
// Four consecutive 16-bit elements from location x (even) on, as the pairs
// (x, x+2) and (x+4, x+6): the three aligned dwords that hold them, shifted
// into place (by 0 or 2 bytes, from the location's low two bits).
template <bool LDS>
__device__ __forceinline__ void mf_da_get4_pk(const unsigned char* gb, uint32_t x, uint32_t& lo, uint32_t& hi)
{
    const auto w = mf_da_dw<LDS>(gb, x);
    const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
    lo = __builtin_amdgcn_alignbyte(w1, w0, x);
    hi = __builtin_amdgcn_alignbyte(w2, w1, x);
}

// Merge chunk: co-rank of rank r0 in (A window, B window), A first on ties,
// over a range of fewer than 2^steps positions; then the chunk's nvalid
// outputs, four per step. A step reads A[ia..ia+3] and B[ib..ib+3]
// (independent loads, one dependent round trip per four outputs): the four
// smallest of the eight are min(A[ia+i], B[ib+3-i]) for i = 0..3 (a
// half-cleaner), element i coming from A exactly when A[ia+i] <= B[ib+3-i];
// a bitonic sort of four puts them in order. The
// elements after each input window are sentinels or list elements ranked
// after every output this chunk must produce, so no step tests for an
// exhausted input; the at most three outputs of the last step past nvalid
// land in the list's sentinel slots, which the lane of the merge's last chunk
// rewrites afterwards. Chunk outputs start at multiples of four elements, so
// every step writes one aligned run of four. CLAMP keeps the A index at the
// window end: needed when data can equal the sentinel value (8-bit data in
// 8-bit elements, 16-bit and 32-bit data), not for 8-bit data held in 16-bit
// elements (the global-memory form).
template <class E, bool CLAMP, bool LDS>
__device__ __forceinline__ void mf_da_merge(E* __restrict__ gl, const uint4 d)
{
    constexpr uint32_t kMask = (1u << 18) - 1;
    constexpr uint32_t kMax = (uint32_t)(E)~(E)0;
    const int ao = (int)(d.x & kMask), bo = (int)(d.y & kMask);
    const E* __restrict__ A = gl + ao;
    const E* __restrict__ B = gl + bo;
    const int na = (int)(d.x >> 18), nb = (int)(d.y >> 18);
    const int oo = (int)(d.z & kMask);
    const int nvalid = (int)(d.z >> 18);
    const int r0 = (int)(d.w & kMask), steps = (int)((d.w >> 18) & 15u);
    // co-rank: pos = lo + #{t in [lo, hi): A[t] <= B[r0-1-t]} (a prefix, the
    // windows being sorted), by halving steps. A probe past the range reads
    // A[hi-1] instead; when that one is taken every position is, and pos
    // becomes hi, the answer. Extra steps at the top (2^s above the range)
    // leave pos unchanged, so the wave runs the largest step count of its
    // lanes as a uniform loop: its first active lane holds it, the chunks of
    // a round being ordered by decreasing step count.
    const int hi = min(r0, na);
    int pos = max(0, r0 - nb);
    const E* __restrict__ Bm = B + (r0 - 1);
    const int sw = __builtin_amdgcn_readfirstlane(steps);
    for (int s = sw - 1; s >= 0; --s) {
        const int tc = min(pos + (1 << s) - 1, hi - 1);
        const uint32_t av = A[tc], bv = Bm[-tc];
        pos = av <= bv ? tc + 1 : pos;
    }
    const int ia = pos;
    if constexpr (sizeof(E) == 1) {
        // 8-bit elements: the 16-bit step on the widened pairs, heads and
        // output as LDS byte addresses. The half-cleaner pairs (a0,a1) with
        // (b3,b2) and (a2,a3) with (b1,b0); a halve's 0/1 "A element larger"
        // flags summed over both pairs give g in {0,1,2} per half, and the
        // number of A elements taken, (2-g.lo) + (2-g.hi), is v_sad_u16 of g
        // against (2,2), added to the A head in the same instruction. The
        // bitonic sort's second stage compares (x0,x2) with (x1,x3), regrouped
        // by v_perm, and the narrowing interleaves its minima and maxima.
        // The B head advances by the B elements taken, g.lo + g.hi (v_sad_u16
        // against 0). When the clamp pulls the A head back, the A elements it
        // took past its window tied with B's head and every later output of
        // the chunk has that value (the elements after a window rank after
        // the chunk's outputs), so the B elements left behind yield the same
        // outputs.
        unsigned char* gb = reinterpret_cast<unsigned char*>(gl);
        uint32_t xa = mf_da_addr<LDS>(gb, A) + (uint32_t)ia;
        const uint32_t xend = mf_da_addr<LDS>(gb, A) + (uint32_t)na;
        uint32_t xo = mf_da_addr<LDS>(gb, gl + oo);
        const uint32_t xo_end = xo + (uint32_t)nvalid;
        uint32_t xb = mf_da_addr<LDS>(gb, B) + (uint32_t)(r0 - ia);
        for (; xo < xo_end; xo += 4) {
            uint32_t a01, a23, r32, r10;
            mf_da_get4_u8<LDS>(gb, xa, a01, a23);
            mf_da_get4_u8_rev<LDS>(gb, xb, r32, r10);
            const uint32_t c01 = mf_pk_min(a01, r32), c23 = mf_pk_min(a23, r10);
            const uint32_t g = mf_pk_gt01(a01, r32) + mf_pk_gt01(a23, r10);
            const uint32_t x01 = mf_pk_min(c01, c23), x23 = mf_pk_max(c01, c23);
            const uint32_t p02 = __builtin_amdgcn_perm(x23, x01, 0x05040100u);
            const uint32_t p13 = __builtin_amdgcn_perm(x23, x01, 0x07060302u);
            const uint32_t mn = mf_pk_min(p02, p13), mx = mf_pk_max(p02, p13);
            mf_da_put<LDS>(gb, xo, __builtin_amdgcn_perm(mx, mn, 0x06020400u));
            xa = __builtin_amdgcn_sad_u16(g, 0x00020002u, xa);
            if constexpr (CLAMP) xa = min(xa, xend);
            xb = __builtin_amdgcn_sad_u16(g, 0u, xb);
        }
    } else if constexpr (sizeof(E) == 2) {
        // the step on pairs, as for 8-bit elements: (a0,a1) meets (b3,b2) and
        // (a2,a3) meets (b1,b0); heads and output as LDS byte addresses, two
        // bytes per element, so the flags are doubled before v_sad_u16 adds
        // twice the number of A elements taken to the A head (and twice the
        // B elements taken to the B head)
        unsigned char* gb = reinterpret_cast<unsigned char*>(gl);
        uint32_t xa = mf_da_addr<LDS>(gb, A) + 2u * (uint32_t)ia;
        const uint32_t xend = mf_da_addr<LDS>(gb, A) + 2u * (uint32_t)na;
        uint32_t xo = mf_da_addr<LDS>(gb, gl + oo);
        const uint32_t xo_end = xo + 2u * (uint32_t)nvalid;
        uint32_t xb = mf_da_addr<LDS>(gb, B) + 2u * (uint32_t)(r0 - ia);
        for (; xo < xo_end; xo += 8) {
            uint32_t a01, a23, b01, b23;
            mf_da_get4_pk<LDS>(gb, xa, a01, a23);
            mf_da_get4_pk<LDS>(gb, xb, b01, b23);
            const uint32_t r32 = mf_swap16(b23), r10 = mf_swap16(b01);
            const uint32_t c01 = mf_pk_min(a01, r32), c23 = mf_pk_min(a23, r10);
            const uint32_t g2 = (mf_pk_gt01(a01, r32) + mf_pk_gt01(a23, r10)) << 1;
            // bitonic sort of four
            const uint32_t x01 = mf_pk_min(c01, c23), x23 = mf_pk_max(c01, c23);
            const uint32_t p02 = __builtin_amdgcn_perm(x23, x01, 0x05040100u);
            const uint32_t p13 = __builtin_amdgcn_perm(x23, x01, 0x07060302u);
            const uint32_t mn = mf_pk_min(p02, p13), mx = mf_pk_max(p02, p13);
            mf_da_put<LDS>(gb, xo, mf_u32x2{__builtin_amdgcn_perm(mx, mn, 0x05040100u),
                                            __builtin_amdgcn_perm(mx, mn, 0x07060302u)});
            xa = __builtin_amdgcn_sad_u16(g2, 0x00040004u, xa);
            if constexpr (CLAMP) xa = min(xa, xend);
            xb = __builtin_amdgcn_sad_u16(g2, 0u, xb);
        }
    } else {
        // 32-bit elements, heads and output as locations (four bytes per
        // element); the number of A elements taken counted by a compare and
        // add-with-carry chain
        unsigned char* gb = reinterpret_cast<unsigned char*>(gl);
        uint32_t xa = mf_da_addr<LDS>(gb, A) + 4u * (uint32_t)ia;
        const uint32_t xend = mf_da_addr<LDS>(gb, A) + 4u * (uint32_t)na;
        uint32_t xo = mf_da_addr<LDS>(gb, gl + oo);
        const uint32_t xo_end = xo + 4u * (uint32_t)nvalid;
        const uint32_t F = mf_da_addr<LDS>(gb, B) + 4u * (uint32_t)r0 + mf_da_addr<LDS>(gb, A) - xo;
        uint32_t xb = xo + F - xa;
        for (; xo < xo_end; xo += 16) {
            uint32_t a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = mf_da_get<LDS, uint32_t>(gb, xa + 4u * i);
                b[i] = mf_da_get<LDS, uint32_t>(gb, xb + 4u * i);
            }
            const uint32_t c0 = min(a[0], b[3]), c1 = min(a[1], b[2]), c2 = min(a[2], b[1]), c3 = min(a[3], b[0]);
            const uint32_t nA = mf_count_le4(a[0], b[3], a[1], b[2], a[2], b[1], a[3], b[0]);
            // bitonic sort of four
            const uint32_t x0 = min(c0, c2), x2 = max(c0, c2);
            const uint32_t x1 = min(c1, c3), x3 = max(c1, c3);
            mf_da_put<LDS>(gb, xo, mf_u32x4{min(x0, x1), max(x0, x1), min(x2, x3), max(x2, x3)});
            xa += 4u * nA;
            if constexpr (CLAMP) xa = min(xa, xend);
            xb = xo + 16u + F - xa;
        }
    }
    if (d.w & (1u << 22)) {
#pragma unroll
        for (int i = 0; i < MF_DA_SENT; ++i) gl[oo + nvalid + i] = (E)kMax;
    }
}

// Footprints of G root tiles (bx*G + t, by) -> arenas gl + t*arena, after
// the guard, row-major fw x fh (replicate border); the guard's last MF_DA_SENT slots of
// each arena hold the sentinel. Work-group-wide; no barrier.
template <class E>
__device__ __forceinline__ void
mf_da_load(E* __restrict__ gl, const unsigned char* __restrict__ src, int H, int W, long long pitch, int dtype,
           const MfDaArgs& a, int G, int bx, int by)
{
    constexpr uint32_t kMax = (uint32_t)(E)~(E)0;
    const int tw = a.tw, th = a.th, arena = a.arena;
    const int rx = (a.k - 1) / 2, ry = (a.kh - 1) / 2;
    const int fw = a.k + tw - 1, fh = a.kh + th - 1;
    const int Y0 = by * th;
    for (int i = threadIdx.x; i < G * fw * fh; i += kDaThreads) {
        const int t = i / (fw * fh), e = i - t * fw * fh;
        const int y = e / fw, x = e - y * fw;
        const int gy = min(max(Y0 - ry + y, 0), H - 1);
        const int gx = min(max((bx * G + t) * tw - rx + x, 0), W - 1);
        const unsigned char* row = src + (long long)gy * pitch;
        uint32_t v;
        if (dtype == MF_U8) v = row[gx];
        else if (dtype == MF_U16) v = ((const uint16_t*)row)[gx];
        else {
            v = ((const uint32_t*)row)[gx];
            if (dtype == MF_F32) v = mf_da_f32_to_key(v);
        }
        gl[t * arena + MF_DA_GUARD + e] = (E)v;
    }
    if (threadIdx.x < G * MF_DA_SENT)
        gl[(threadIdx.x / MF_DA_SENT) * arena + MF_DA_GUARD - MF_DA_SENT + threadIdx.x % MF_DA_SENT] = (E)kMax;
}

// Rounds [r0, r1) of the schedule on one arena, lane lt of the L lanes that
// share it; a work-group barrier after every round.
// One item: a sort or a merge chunk.
template <class E, bool CLAMP, bool LDS>
__device__ __forceinline__ void mf_da_item(E* __restrict__ gl, const uint4 d)
{
    if (d.w & 0x80000000u) {
        switch (d.w & 63u) {
        case 1: mf_da_sort<E, 1, LDS>(gl, d); break;
        case 2: mf_da_sort<E, 2, LDS>(gl, d); break;
        case 4: mf_da_sort<E, 4, LDS>(gl, d); break;
        case 8: mf_da_sort<E, 8, LDS>(gl, d); break;
        case 16: mf_da_sort<E, 16, LDS>(gl, d); break;
        default: mf_da_sort<E, 32, LDS>(gl, d); break;
        }
    } else {
        mf_da_merge<E, CLAMP, LDS>(gl, d);
    }
}

template <class E, bool CLAMP, bool LDS = true>
__device__ __forceinline__ void mf_da_rounds(E* __restrict__ gl, const MfDaArgs& a, int r0, int r1, int lt, int L)
{
    const uint32_t* __restrict__ blob = a.blob;
    const uint4* __restrict__ items = reinterpret_cast<const uint4*>(blob + a.c_off);
    const uint32_t* __restrict__ rounds = blob + a.r_off;
    for (int rd = r0; rd < r1; ++rd) {
        const int c1 = (int)rounds[rd + 1];
        for (int c = (int)rounds[rd] + lt; c < c1; c += L)
            mf_da_item<E, CLAMP, LDS>(gl, items[c]);
        __syncthreads();
    }
}

// The lane's index in its wave, computed afresh where it is written (the
// asm is volatile, so it is not hoisted and kept live across a loop).
__device__ __forceinline__ int mf_lane_now()
{
    uint32_t lo, r;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0" : "=v"(lo));
    asm volatile("v_mbcnt_hi_u32_b32 %0, -1, %1" : "=v"(r) : "v"(lo));
    return (int)r;
}

// As mf_da_rounds, for lane groups of whole waves (L a multiple of 64): lane
// lt = lw + the lane's index in its wave, lw the same on every lane of a wave.
// The item loop runs on the wave's first item (a scalar), and the lane's own
// item is that plus its lane index, recomputed per item: no per-lane loop
// state stays live across the sorting networks.
template <class E, bool CLAMP>
__device__ __forceinline__ void mf_da_rounds_wave(E* __restrict__ gl, const MfDaArgs& a, int lw, int L)
{
    const uint32_t* __restrict__ blob = a.blob;
    const uint4* __restrict__ items = reinterpret_cast<const uint4*>(blob + a.c_off);
    const uint32_t* __restrict__ rounds = blob + a.r_off;
    for (int rd = 0; rd < a.nrounds; ++rd) {
        // item range as scalars (read once per round)
        const int c0 = __builtin_amdgcn_readfirstlane((int)rounds[rd]);
        const int c1 = __builtin_amdgcn_readfirstlane((int)rounds[rd + 1]);
        for (int cw = c0 + lw; cw < c1; cw += L) {
            const int c = cw + mf_lane_now();
            if (c < c1) mf_da_item<E, CLAMP, true>(gl, items[c]);
        }
        __syncthreads();
    }
}

// All rounds on the LDS arena of lane group gi. When a group spans whole
// waves (L >= 64) the arena base is the same on every lane of a wave and is
// kept in a scalar register, and for 8- and 16-bit elements so is the item
// loop (measured: 1.04-1.07x slower for 32-bit elements); otherwise both
// are per lane.
template <class E, bool CLAMP>
__device__ __forceinline__ void mf_da_rounds_lds(E* __restrict__ lds, const MfDaArgs& a, int gi, int lt, int L)
{
    if (L >= 64) {
        const int gu = __builtin_amdgcn_readfirstlane(gi);
        if constexpr (sizeof(E) < 4)
            mf_da_rounds_wave<E, CLAMP>(lds + gu * a.arena, a, __builtin_amdgcn_readfirstlane(lt - (int)__lane_id()),
                                        L);
        else
            mf_da_rounds<E, CLAMP>(lds + gu * a.arena, a, 0, a.nrounds, lt, L);
    } else
        mf_da_rounds<E, CLAMP>(lds + gi * a.arena, a, 0, a.nrounds, lt, L);
}

// Medians of G root tiles (bx*G + t, by) from their arenas to dst.
template <class E>
__device__ __forceinline__ void
mf_da_store(const E* __restrict__ gl, unsigned char* __restrict__ dst, int H, int W, long long pitch, int dtype,
            const MfDaArgs& a, int G, int bx, int by)
{
    const int tw = a.tw, th = a.th, arena = a.arena;
    const int Y0 = by * th;
    const uint32_t* outs = a.blob + a.o_off;
    for (int p = threadIdx.x; p < G * tw * th; p += kDaThreads) {
        const int t = p / (tw * th), e = p - t * tw * th;
        const int y = Y0 + e / tw, x = (bx * G + t) * tw + e % tw;
        if (y >= H || x >= W) continue;
        unsigned char* row = dst + (long long)y * pitch;
        const uint32_t v = (uint32_t)gl[t * arena + outs[e]];
        if (dtype == MF_U8) row[x] = (unsigned char)v;
        else if (dtype == MF_U16) ((uint16_t*)row)[x] = (uint16_t)v;
        else ((uint32_t*)row)[x] = (dtype == MF_F32) ? mf_da_key_to_f32(v) : v;
    }
}

// G root tiles (bx*G + g, by) of one image, schedule `a`, G = a.groups, in
// LDS. The work-group's lanes form G groups of kDaThreads/G lanes; group g
// owns tile g and runs every round's items for it (small tiles, whose rounds
// have few items, fill the work-group this way). LDS holds G arenas of
// `arena` elements.
// Tile of work-group b of n in one plane. Work-groups are dealt to the 8
// XCDs in turn (b % 8), each with its own L2; this hands XCD x the x-th
// contiguous eighth of the row-major tiles, in order, so horizontally
// adjacent tiles (which share all but t_w columns of their footprints) run on
// the same XCD one after the other and the rows above and below are read
// shortly before. A bijection of [0, n) for any n.
__device__ __forceinline__ int mf_da_xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

template <class E, bool CLAMP>
__device__ __forceinline__ void
mf_da_block(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
            long long pitch, int dtype, const MfDaArgs& a, int bx, int by)
{
    extern __shared__ __align__(16) unsigned char mf_da_lds[];
    E* lds = reinterpret_cast<E*>(mf_da_lds);
    const int G = a.groups, L = kDaThreads / G;
    const int gi = threadIdx.x / L, lt = threadIdx.x - gi * L;
    mf_da_load<E>(lds, src, H, W, pitch, dtype, a, G, bx, by);
    __syncthreads();
    mf_da_rounds_lds<E, CLAMP>(lds, a, gi, lt, L);
    mf_da_store<E>(lds, dst, H, W, pitch, dtype, a, G, bx, by);
}

// WAVES: the register budget the compiler is asked for (waves per SIMD; 0 =
// none). 8- and 16-bit arenas small enough for four work-groups per CU take
// the eight-wave budget (64 VGPRs: the sorting networks spill a little), the
// others the default, which keeps six waves.
template <class E, bool CLAMP, int WAVES = 0>
__global__ void __launch_bounds__(kDaThreads) __attribute__((amdgpu_waves_per_eu(WAVES ? WAVES : 1)))
mf_da_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
             long long pitch, long long plane_stride, int dtype, MfDaArgs a, int ntx)
{
    const long long po = (long long)blockIdx.y * plane_stride;   // plane = blockIdx.y
    const int t = mf_da_xcd_tile((int)blockIdx.x, (int)gridDim.x);
    mf_da_block<E, CLAMP>(src + po, dst + po, H, W, pitch, dtype, a, t % ntx, t / ntx);
}

// Batched form, persistent: a resident-sized grid walks the nblocks blocks
// of every image of a job table (same k, tile and element size), work-group
// w taking blocks w, w + gridDim.x, ...; image found by binary search over
// the first block indices.
template <class E, bool CLAMP>
__global__ void __launch_bounds__(kDaThreads)
mf_da_kernel_batched(const MfJob* __restrict__ jobs, int njobs, int nblocks, MfDaArgs a)
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
        mf_da_block<E, CLAMP>(j.src, j.dst, j.H, j.W, j.pitch, j.dtype, a, lb % j.nbx, lb / j.nbx);
        __syncthreads();   // the next block reuses the LDS
    }
}

// Global-memory multi-pass form (Section 5.3: passes of two recursion levels
// over a slice of tiles, lists in device memory). One work-group per tile
// of the slice [tile0, tile0 + gridDim.x); work-group b keeps the tile's
// lists in workspace slot b (arena elements) from pass to pass. A launch
// runs rounds [r0, r1): the first pass also loads the footprint, the last
// one stores the medians. Tiles are numbered plane by plane, row-major.
template <class E, bool CLAMP>
__global__ void __launch_bounds__(kDaThreads)
mf_dag_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
              long long pitch, long long plane_stride, int dtype, MfDaArgs a, int ntx, int tiles_per_plane,
              long long tile0, E* __restrict__ ws, int r0, int r1, int first, int last)
{
    const long long tile = tile0 + blockIdx.x;
    const long long plane = tile / tiles_per_plane;
    const int t = (int)(tile - plane * tiles_per_plane);
    const int bx = t % ntx, by = t / ntx;
    E* gl = ws + (size_t)blockIdx.x * (size_t)a.arena;
    if (first) {
        mf_da_load<E>(gl, src + plane * plane_stride, H, W, pitch, dtype, a, 1, bx, by);
        __syncthreads();
    }
    mf_da_rounds<E, CLAMP, false>(gl, a, r0, r1, threadIdx.x, kDaThreads);
    if (last) mf_da_store<E>(gl, dst + plane * plane_stride, H, W, pitch, dtype, a, 1, bx, by);
}

// 3-D box median (the hierarchical recursion with a third axis): G root tiles
// of tw x th x tz voxels per work-group, side by side along x (G = a.groups
// lane groups of kDaThreads/G lanes, small tiles filling the work-group),
// each tile's (k+tw-1) x (kh+th-1) x (kz+tz-1) footprint in its own LDS arena
// (each axis clamped), the schedule's rounds, and the tiles' medians stored.
// Rows are pitch bytes apart, slices slice bytes apart; work-group b covers
// tile columns (b % ntx)*G .. +G-1, row b / ntx % nty, slab b / (ntx*nty).
template <class E, bool CLAMP>
__global__ void __launch_bounds__(kDaThreads)
mf_da3_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int D, int H, int W,
              long long pitch, long long slice, int dtype, MfDaArgs a, int ntx, int nty)
{
    extern __shared__ __align__(16) unsigned char mf_da_lds[];
    constexpr uint32_t kMax = (uint32_t)(E)~(E)0;
    E* lds = reinterpret_cast<E*>(mf_da_lds);
    const int G = a.groups, L = kDaThreads / G;
    const int gi = threadIdx.x / L, lt = threadIdx.x - gi * L;
    const int b = mf_da_xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
    const int fw = a.k + a.tw - 1, fh = a.kh + a.th - 1, fd = a.kz + a.tz - 1;
    const int fp = fw * fh * fd;
    const int rx = (a.k - 1) / 2, ry = (a.kh - 1) / 2, rz = (a.kz - 1) / 2;
    const int Y0 = by * a.th - ry, Z0 = bz * a.tz - rz;
    for (int i = threadIdx.x; i < G * fp; i += kDaThreads) {
        const int t = i / fp, e = i - t * fp;
        const int z = e / (fw * fh), r = e - z * fw * fh;
        const int y = r / fw, x = r - y * fw;
        const int gz = min(max(Z0 + z, 0), D - 1), gy = min(max(Y0 + y, 0), H - 1);
        const int gx = min(max((bx * G + t) * a.tw - rx + x, 0), W - 1);
        const unsigned char* row = src + (long long)gz * slice + (long long)gy * pitch;
        uint32_t v;
        if (dtype == MF_U8) v = row[gx];
        else if (dtype == MF_U16) v = ((const uint16_t*)row)[gx];
        else {
            v = ((const uint32_t*)row)[gx];
            if (dtype == MF_F32) v = mf_da_f32_to_key(v);
        }
        lds[t * a.arena + MF_DA_GUARD + e] = (E)v;
    }
    if (threadIdx.x < G * MF_DA_SENT)
        lds[(threadIdx.x / MF_DA_SENT) * a.arena + MF_DA_GUARD - MF_DA_SENT + threadIdx.x % MF_DA_SENT] = (E)kMax;
    __syncthreads();
    mf_da_rounds_lds<E, CLAMP>(lds, a, gi, lt, L);
    const uint32_t* outs = a.blob + a.o_off;
    const int tv = a.tw * a.th * a.tz;
    for (int q = threadIdx.x; q < G * tv; q += kDaThreads) {
        const int t = q / tv, p = q - t * tv;
        const int pz = p / (a.tw * a.th), r = p - pz * a.tw * a.th;
        const int py = r / a.tw, px = r - py * a.tw;
        const int z = bz * a.tz + pz, y = by * a.th + py, x = (bx * G + t) * a.tw + px;
        if (z >= D || y >= H || x >= W) continue;
        unsigned char* row = dst + (long long)z * slice + (long long)y * pitch;
        const uint32_t v = (uint32_t)lds[t * a.arena + outs[p]];
        if (dtype == MF_U8) row[x] = (unsigned char)v;
        else if (dtype == MF_U16) ((uint16_t*)row)[x] = (uint16_t)v;
        else ((uint32_t*)row)[x] = (dtype == MF_F32) ? mf_da_key_to_f32(v) : v;
    }
}

namespace {

// 3-D kernel pointers by value class: bytes for 8-bit data (sentinel 0xff,
// clamped), 16-bit elements for 16-bit data, 32-bit elements for 32-bit data
const void* da3_kernel_for_dtype(int dtype)
{
    if (dtype == MF_U8) return (const void*)mf_da3_kernel<uint8_t, true>;
    if (dtype == MF_U16) return (const void*)mf_da3_kernel<uint16_t, true>;
    return (const void*)mf_da3_kernel<uint32_t, true>;
}

// 8-bit data: bytes in LDS (sentinel 0xff, equal to the largest data value,
// hence the clamped kernel).
constexpr size_t kDaLdsFourPerCu = 160 * 1024 / 4;

// the one-plane 8- and 16-bit kernels with the eight-wave register budget
const void* da_kernel_w8(int dtype)
{
    return dtype == MF_U8 ? (const void*)mf_da_kernel<uint8_t, true, 8> : (const void*)mf_da_kernel<uint16_t, true, 8>;
}

const void* da_kernel_for_dtype(int dtype, bool batched)
{
    if (dtype == MF_U8)
        return batched ? (const void*)mf_da_kernel_batched<uint8_t, true> : (const void*)mf_da_kernel<uint8_t, true>;
    if (dtype == MF_U16)
        return batched ? (const void*)mf_da_kernel_batched<uint16_t, true> : (const void*)mf_da_kernel<uint16_t, true>;
    return batched ? (const void*)mf_da_kernel_batched<uint32_t, true> : (const void*)mf_da_kernel<uint32_t, true>;
}

}  // namespace

namespace {

// kh = 0: the square k x k window; form 0 = any round mode (the first
// entry, the default), 1 = rounds per recursion level, 2 = over the whole
// schedule
const DaEntry* da_find(int dtype, int k, int tw, int th, int group, int kh = 0, int form = 0)
{
    const int es = (dtype == MF_U8 || dtype == MF_U16) ? 2 : 4;
    if (kh == 0) kh = k;
    for (int i = 0; i < kDaCount; ++i) {
        const DaEntry& e = kDaTable[i];
        if (e.mem == 0 && e.kz == 1 && e.k == k && e.kh == kh && e.es == es && (tw == 0 || e.tw == tw) &&
            (th == 0 || e.th == th) && (group == 0 || e.tiles == group) && (form == 0 || e.mode == form - 1))
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
        for (int dt = MF_U8; dt <= MF_U32; ++dt)
            for (int bt = 0; bt < 3; ++bt) {
                const void* fn = bt == 2 ? da3_kernel_for_dtype(dt) : da_kernel_for_dtype(dt, bt != 0);
                e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
                if (e != hipSuccess) return e;
            }
        for (int dt = MF_U8; dt <= MF_U16; ++dt) {
            e = hipFuncSetAttribute(da_kernel_w8(dt), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
        }
        g_da_blob_dev[dev] = (const uint32_t*)p;
    }
    *out = g_da_blob_dev[dev];
    return hipSuccess;
}

}  // namespace

bool mf_da_supports(int dtype, int k, int tw, int th, int group, int kh, int form)
{
    return da_find(dtype, k, tw, th, group, kh, form) != nullptr;
}

int mf_da_rect_max_side() { return MF_DA_RECT_MAX_SIDE; }

void mf_da_default_tile(int dtype, int k, int* tw, int* th, int* group, int kh, int* form)
{
    const DaEntry* e = da_find(dtype, k, 0, 0, 0, kh);
    *tw = e ? e->tw : 0;
    *th = e ? e->th : 0;
    *group = e ? e->tiles : 0;
    if (form) *form = e ? e->mode + 1 : 0;
}

int mf_da_list(int dtype, int k, int* tw, int* th, int* group, int cap, int* form)
{
    const int es = (dtype == MF_U8 || dtype == MF_U16) ? 2 : 4;
    int n = 0;
    for (int i = 0; i < kDaCount; ++i) {
        const DaEntry& e = kDaTable[i];
        if (e.mem != 0 || e.kz != 1 || e.k != k || e.kh != k || e.es != es) continue;
        if (n < cap) {
            tw[n] = e.tw;
            th[n] = e.th;
            group[n] = e.tiles;
            if (form) form[n] = e.mode + 1;
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
    a.kz = e->kz;
    a.tz = e->tz;
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
                        long long pitch, int dtype, int k, int tw, int th, int group, hipStream_t stream, int kh,
                        int form)
{
    const DaEntry* e = da_find(dtype, k, tw, th, group, kh, form);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    MfDaArgs a = da_args(e, blob);
    const int bw = e->tw * e->tiles * e->groups;     // pixels of a work-group along x
    const int ntx = (W + bw - 1) / bw, nty = (H + e->th - 1) / e->th;
    if ((long long)ntx * nty > 0x7fffffffLL) return hipErrorInvalidConfiguration;   // grid.x limit
    const size_t lds = (size_t)e->arena * (dtype == MF_U8 ? 1 : e->es) * e->tiles * e->groups;
    for (int p0 = 0; p0 < planes; p0 += 65535) {     // grid rows are planes
        const int np = planes - p0 < 65535 ? planes - p0 : 65535;
        const unsigned char* s8 = (const unsigned char*)src + p0 * plane_stride;
        unsigned char* d8 = (unsigned char*)dst + p0 * plane_stride;
        void* args[] = {&s8, &d8, &H, &W, &pitch, &plane_stride, &dtype, &a, (void*)&ntx};
        const void* fn = (dtype == MF_U8 || dtype == MF_U16) && lds <= kDaLdsFourPerCu ? da_kernel_w8(dtype)
                                                                                      : da_kernel_for_dtype(dtype, false);
        err = hipLaunchKernel(fn, dim3(ntx * nty, np), dim3(kDaThreads), args, lds, stream);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t mf_da_batched(int dtype, int k, int tw, int th, int group, MfBatchedKernel* kern, MfDaArgs* args,
                         int form)
{
    const DaEntry* e = da_find(dtype, k, tw, th, group, 0, form);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    *args = da_args(e, blob);
    kern->fn = da_kernel_for_dtype(dtype, true);
    kern->threads = kDaThreads;
    kern->lds = (size_t)e->arena * (dtype == MF_U8 ? 1 : e->es) * e->tiles * e->groups;
    kern->bw = e->tw * e->tiles * e->groups;
    kern->bh = e->th;
    return hipSuccess;
}

// ---- Global-memory multi-pass form ------------------------------------

namespace {

const DaEntry* dag_find(int dtype, int k, int tw, int th)
{
    const int es = (dtype == MF_U8 || dtype == MF_U16) ? 2 : 4;
    for (int i = 0; i < kDaCount; ++i) {
        const DaEntry& e = kDaTable[i];
        if (e.mem == 1 && e.kz == 1 && e.k == k && e.kh == k && e.es == es && (tw == 0 || e.tw == tw) &&
            (th == 0 || e.th == th))
            return &e;
    }
    // any schedule of this element size and tile also runs from the workspace
    if (tw && th) {
        for (int i = 0; i < kDaCount; ++i) {
            const DaEntry& e = kDaTable[i];
            if (e.kz == 1 && e.k == k && e.kh == k && e.es == es && e.tw == tw && e.th == th && e.groups == 1)
                return &e;
        }
    }
    return nullptr;
}

const void* dag_kernel_for_dtype(int dtype)
{
    if (dtype == MF_U8) return (const void*)mf_dag_kernel<uint16_t, false>;
    if (dtype == MF_U16) return (const void*)mf_dag_kernel<uint16_t, true>;
    return (const void*)mf_dag_kernel<uint32_t, true>;
}

long long dag_slot_bytes(const DaEntry* e) { return (((long long)e->arena * e->es) + 255) / 256 * 256; }

}  // namespace

bool mf_dag_supports(int dtype, int k, int tw, int th) { return dag_find(dtype, k, tw, th) != nullptr; }

bool mf_dag_workspace(int dtype, int k, int tw, int th, long long planes, int H, int W, long long* slot_bytes,
                      long long* all_bytes, int* used_tw, int* used_th)
{
    const DaEntry* e = dag_find(dtype, k, tw, th);
    if (!e) return false;
    const long long ntx = (W + e->tw - 1) / e->tw, nty = (H + e->th - 1) / e->th;
    *slot_bytes = dag_slot_bytes(e);
    *all_bytes = *slot_bytes * ntx * nty * planes;
    *used_tw = e->tw;
    *used_th = e->th;
    return true;
}

int mf_dag_passes(int dtype, int k, int tw, int th)
{
    const DaEntry* e = dag_find(dtype, k, tw, th);
    if (!e) return 0;
    const uint32_t* phase = reinterpret_cast<const uint32_t*>(mf_da_blob_host) + e->p_off;
    int n = 0;
    for (int r = 0; r < e->nrounds; ++r)
        if (r == 0 || phase[r] / 2 != phase[r - 1] / 2) ++n;
    return n;
}

hipError_t mf_dag_launch(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                         long long pitch, int dtype, int k, int tw, int th, void* ws, long long ws_bytes,
                         hipStream_t stream)
{
    const DaEntry* e = dag_find(dtype, k, tw, th);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    MfDaArgs a = da_args(e, blob);
    a.groups = 1;
    const int ntx = (W + e->tw - 1) / e->tw, nty = (H + e->th - 1) / e->th;
    const int per_plane = ntx * nty;
    const long long total = (long long)per_plane * planes;
    const long long slot = dag_slot_bytes(e);
    long long slice = ws_bytes / slot;
    if (slice < 1) return hipErrorInvalidValue;
    if (slice > total) slice = total;
    if (slice > 0x7fffffffLL) slice = 0x7fffffffLL;
    // passes: consecutive rounds of two recursion levels each (the
    // initialisation is level 0)
    const uint32_t* phase = reinterpret_cast<const uint32_t*>(mf_da_blob_host) + e->p_off;
    int bounds[64];
    int nb = 0;
    for (int r = 0; r < e->nrounds && nb < 63; ++r)
        if (r == 0 || phase[r] / 2 != phase[r - 1] / 2) bounds[nb++] = r;
    bounds[nb] = e->nrounds;
    const void* fn = dag_kernel_for_dtype(dtype);
    for (long long t0 = 0; t0 < total; t0 += slice) {
        const unsigned grid = (unsigned)(total - t0 < slice ? total - t0 : slice);
        for (int p = 0; p < nb; ++p) {
            int r0 = bounds[p], r1 = bounds[p + 1], first = p == 0, last = p == nb - 1;
            void* args[] = {&src, &dst, &H, &W, &pitch, &plane_stride, &dtype, &a, (void*)&ntx, (void*)&per_plane,
                            &t0, &ws, &r0, &r1, &first, &last};
            err = hipLaunchKernel(fn, dim3(grid), dim3(kDaThreads), args, 0, stream);
            if (err != hipSuccess) return err;
        }
    }
    return hipSuccess;
}

// ---- 3-D boxes --------------------------------------------------------

namespace {

const DaEntry* da3_find(int dtype, int k)
{
    const int es = (dtype == MF_U8 || dtype == MF_U16) ? 2 : 4;
    for (int i = 0; i < kDaCount; ++i) {
        const DaEntry& e = kDaTable[i];
        if (e.kz > 1 && e.k == k && e.kh == k && e.kz == k && e.es == es) return &e;
    }
    return nullptr;
}

}  // namespace

bool mf_da3_supports(int dtype, int k) { return da3_find(dtype, k) != nullptr; }

int mf_da3_max_k()
{
    int m = 0;
    for (int i = 0; i < kDaCount; ++i)
        if (kDaTable[i].kz > 1 && kDaTable[i].kz > m) m = kDaTable[i].kz;
    return m;
}

void mf_da3_tile(int dtype, int k, int* tw, int* th, int* tz)
{
    const DaEntry* e = da3_find(dtype, k);
    *tw = e ? e->tw : 0;
    *th = e ? e->th : 0;
    *tz = e ? e->tz : 0;
}

hipError_t mf_da3_launch(const void* src, void* dst, int D, int H, int W, long long pitch, long long slice, int dtype,
                         int k, hipStream_t stream)
{
    const DaEntry* e = da3_find(dtype, k);
    if (!e) return hipErrorInvalidValue;
    const uint32_t* blob = nullptr;
    hipError_t err = da_blob(&blob);
    if (err != hipSuccess) return err;
    MfDaArgs a = da_args(e, blob);
    const int bw = e->tw * e->groups;     // voxels of a work-group along x
    const int ntx = (W + bw - 1) / bw, nty = (H + e->th - 1) / e->th, ntz = (D + e->tz - 1) / e->tz;
    if ((long long)ntx * nty * ntz > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const size_t lds = (size_t)e->arena * (dtype == MF_U8 ? 1 : e->es) * e->groups;
    void* args[] = {&src, &dst, &D, &H, &W, &pitch, &slice, &dtype, &a, (void*)&ntx, (void*)&nty};
    return hipLaunchKernel(da3_kernel_for_dtype(dtype), dim3(ntx * nty * ntz), dim3(kDaThreads), args, lds, stream);
}
