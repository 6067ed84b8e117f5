// Column-strip form of the data-oblivious filter for k = 3 (root tile 1 x 1,
// Sections 3.3 and 4 of Sugy 2025), built for streaming HBM at small k.
//
// At k = 3 the hierarchy has a single level: every footprint column of three
// values is sorted once (initialisation, shared by the three horizontally
// adjacent windows that contain it) and the median of the window is the
// pruned three-way merge of its three sorted columns, which reduces to
//     med3(max of the column minima, med3 of the column medians,
//          min of the column maxima).
// With v_min3 / v_max3 / v_med3 that is three instructions per sorted column
// and four per output.
//
// Each wave owns a strip of 64 lanes x P pixels (one 8-byte chunk per lane and
// row for 8-bit data, 16 bytes otherwise) and R = 32 output rows. A lane streams the R + 2 input rows of its
// chunk through registers with the next 8 rows always in flight (no LDS, no
// barriers), keeps three rows and a sliding window of three sorted columns,
// and stores each output row as one chunk. The columns just left and
// right of a lane's chunk come from the neighbouring lanes by a lane shuffle;
// lanes 0 and 63 load theirs. A work-group stacks 4 waves vertically.
#include "mf_internal.h"

namespace {

constexpr int kStripRows = 32;     // output rows per wave
constexpr int kStripDepth = 8;     // input rows loaded ahead of their use
constexpr int kStripWaves = 4;     // waves per work-group, stacked vertically

__device__ __forceinline__ uint32_t smin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t smax(uint32_t a, uint32_t b) { return a < b ? b : a; }
__device__ __forceinline__ uint32_t smed3(uint32_t a, uint32_t b, uint32_t c)
{
    return smax(smin(a, b), smin(smax(a, b), c));
}

// float32 bit pattern <-> uint32 key ordered as IEEE totalOrder
__device__ __forceinline__ uint32_t strip_key(uint32_t b) { return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u); }
__device__ __forceinline__ uint32_t strip_unkey(uint32_t k)
{
    return k ^ ((uint32_t)((int32_t)~k >> 31) | 0x80000000u);
}

// A lane's chunk of one row: CB bytes (8 or 16) as CB/4 words.
template <int CB>
struct Chunk {
    uint32_t w[CB / 4];
};

template <int CB>
__device__ __forceinline__ Chunk<CB> chunk_load(const unsigned char* p)
{
    Chunk<CB> q;
    if constexpr (CB == 16) {
        const uint4 v = *(const uint4*)p;
        q.w[0] = v.x; q.w[1] = v.y; q.w[2] = v.z; q.w[3] = v.w;
    } else {
        const uint2 v = *(const uint2*)p;
        q.w[0] = v.x; q.w[1] = v.y;
    }
    return q;
}

template <int CB>
__device__ __forceinline__ void chunk_store(unsigned char* p, const Chunk<CB>& q)
{
    if constexpr (CB == 16) *(uint4*)p = make_uint4(q.w[0], q.w[1], q.w[2], q.w[3]);
    else *(uint2*)p = make_uint2(q.w[0], q.w[1]);
}

template <int ES, int CB>
__device__ __forceinline__ uint32_t strip_elem(const Chunk<CB>& q, int e)
{
    const uint32_t w = q.w[e * ES / 4];
    if constexpr (ES == 1) return (w >> (8 * (e % 4))) & 0xFFu;
    if constexpr (ES == 2) return (w >> (16 * (e % 2))) & 0xFFFFu;
    return w;
}

template <int ES>
__device__ __forceinline__ uint32_t strip_load1(const unsigned char* row, int x)
{
    if constexpr (ES == 1) return row[x];
    if constexpr (ES == 2) return ((const uint16_t*)row)[x];
    return ((const uint32_t*)row)[x];
}

template <int ES>
__device__ __forceinline__ void strip_store1(unsigned char* row, int x, uint32_t v)
{
    if constexpr (ES == 1) row[x] = (unsigned char)v;
    else if constexpr (ES == 2) ((uint16_t*)row)[x] = (uint16_t)v;
    else ((uint32_t*)row)[x] = v;
}

// three-input min / median / max, one VALU instruction each
__device__ __forceinline__ uint32_t vmin3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t vmax3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_max3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t vmed3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

template <int ES, int CB>
__global__ void __launch_bounds__(64 * kStripWaves)
mf_strip3_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
                 long long pitch, long long plane_stride, int dtype, int nbx, int aligned)
{
    src += (long long)blockIdx.y * plane_stride;   // plane = blockIdx.y
    dst += (long long)blockIdx.y * plane_stride;
    constexpr int P = CB / ES;               // pixels per lane
    constexpr int R = kStripRows;
    constexpr int NR = R + 2;                // input rows of a wave
    constexpr int D = kStripDepth;           // input rows in flight ahead of use
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
    const int x0 = bx * 64 * P + lane * P;    // first pixel of this lane's chunk
    const int y0 = (by * kStripWaves + wv) * R;
    if (y0 >= H) return;                      // whole wave; the kernel has no barriers
    const bool key = ES == 4 && dtype == MF_F32;
    // whole-chunk loads: inside the row, or straddling its end on a row
    // that is not the plane's last (the bytes past the row belong to the
    // padding or the next row and are replaced below)
    const bool inside = aligned && x0 + P <= W;
    const bool straddle = aligned && x0 < W && x0 + P > W;
    const bool beyond = x0 >= W;
    const int nvalid = min(W - x0, P);        // pixels of the chunk inside the row
    const bool edge_lane = lane == 0 || lane == 63;
    const int hx = lane == 0 ? max(x0 - 1, 0) : min(x0 + P, W - 1);

    // input row i of the wave is image row y0 - 1 + i (clamped: replicate)
    auto row_ptr = [&](int i) {
        return src + (long long)min(max(y0 - 1 + i, 0), H - 1) * pitch;
    };
    auto load_row = [&](int i, Chunk<CB>& q, uint32_t& h) {
        const unsigned char* row = row_ptr(i);
        const bool last_row = min(max(y0 - 1 + i, 0), H - 1) == H - 1;
        if (inside || (straddle && !last_row)) {
            q = chunk_load<CB>(row + (long long)x0 * ES);
        } else if (beyond) {
            uint32_t v = strip_load1<ES>(row, W - 1);
            if constexpr (ES == 1) v *= 0x01010101u;
            if constexpr (ES == 2) v *= 0x00010001u;
#pragma unroll
            for (int j = 0; j < CB / 4; ++j) q.w[j] = v;
        } else {
            // unaligned buffers, or the plane's last row at the right edge
#pragma unroll
            for (int j = 0; j < CB / 4; ++j) q.w[j] = 0;
#pragma unroll
            for (int e = 0; e < P; ++e)
                q.w[e * ES / 4] |= strip_load1<ES>(row, min(x0 + e, W - 1)) << (8 * ((e * ES) % 4));
        }
        h = 0;
        if (edge_lane) h = strip_load1<ES>(row, hx);
    };

    // ring of the next D input rows, loaded D rows ahead of their use
    Chunk<CB> ring[D];
    uint32_t hring[D];
#pragma unroll
    for (int i = 0; i < D && i < NR; ++i) load_row(i, ring[i], hring[i]);

    // input row i as P + 2 keys: [0] = column x0-1, [1..P] = the chunk,
    // [P+1] = column x0+P; pixels past the row's end repeat column W-1
    auto unpack = [&](int i, uint32_t* v) {
        const Chunk<CB> q = ring[i % D];
        const uint32_t hq = hring[i % D];
        if (i + D < NR) load_row(i + D, ring[i % D], hring[i % D]);
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const uint32_t u = strip_elem<ES, CB>(q, e);
            v[e + 1] = key ? strip_key(u) : u;
        }
        if (straddle) {
            uint32_t lastv = v[1];
#pragma unroll
            for (int e = 1; e < P; ++e) lastv = e < nvalid ? v[e + 1] : lastv;
#pragma unroll
            for (int e = 1; e < P; ++e) v[e + 1] = e < nvalid ? v[e + 1] : lastv;
        }
        const uint32_t left = __shfl_up(v[P], 1), right = __shfl_down(v[1], 1);
        const uint32_t h = key ? strip_key(hq) : hq;
        v[0] = lane == 0 ? h : left;
        v[P + 1] = lane == 63 ? h : right;
    };

    uint32_t a[P + 2], b[P + 2], c[P + 2];
    unpack(0, a);
    unpack(1, b);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        unpack(i + 2, c);
        // sorted columns (initialisation, shared by the three windows) and
        // the pruned three-way merge of each window's columns, on a sliding
        // window of three sorted columns
        uint32_t lo0 = vmin3(a[0], b[0], c[0]), mi0 = vmed3(a[0], b[0], c[0]), hi0 = vmax3(a[0], b[0], c[0]);
        uint32_t lo1 = vmin3(a[1], b[1], c[1]), mi1 = vmed3(a[1], b[1], c[1]), hi1 = vmax3(a[1], b[1], c[1]);
        Chunk<CB> w;
#pragma unroll
        for (int j = 0; j < CB / 4; ++j) w.w[j] = 0;
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const uint32_t lo2 = vmin3(a[e + 2], b[e + 2], c[e + 2]);
            const uint32_t mi2 = vmed3(a[e + 2], b[e + 2], c[e + 2]);
            const uint32_t hi2 = vmax3(a[e + 2], b[e + 2], c[e + 2]);
            uint32_t o = vmed3(vmax3(lo0, lo1, lo2), vmed3(mi0, mi1, mi2), vmin3(hi0, hi1, hi2));
            if (key) o = strip_unkey(o);
            w.w[e * ES / 4] |= o << (8 * ((e * ES) % 4));
            lo0 = lo1; mi0 = mi1; hi0 = hi1;
            lo1 = lo2; mi1 = mi2; hi1 = hi2;
        }
        const int y = y0 + i;
        if (y < H) {
            unsigned char* row = dst + (long long)y * pitch;
            if (inside) {
                chunk_store<CB>(row + (long long)x0 * ES, w);
            } else if (!beyond) {
#pragma unroll
                for (int e = 0; e < P; ++e)
                    if (e < nvalid) strip_store1<ES>(row, x0 + e, strip_elem<ES, CB>(w, e));
            }
        }
#pragma unroll
        for (int e = 0; e < P + 2; ++e) {
            a[e] = b[e];
            b[e] = c[e];
        }
    }
}

template <int ES, int CB>
hipError_t strip3_launch(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                         long long pitch, int dtype, hipStream_t st)
{
    constexpr int span = 64 * (CB / ES);
    const int nbx = (W + span - 1) / span;
    const int nby = (H + kStripRows * kStripWaves - 1) / (kStripRows * kStripWaves);
    // whole-chunk loads and stores need 16-byte aligned rows
    const int aligned = ((uintptr_t)src % 16 == 0 && (uintptr_t)dst % 16 == 0 && pitch % 16 == 0 &&
                         plane_stride % 16 == 0) ? 1 : 0;
    for (int p0 = 0; p0 < planes; p0 += 65535) {     // grid rows are planes
        const int np = planes - p0 < 65535 ? planes - p0 : 65535;
        hipLaunchKernelGGL((mf_strip3_kernel<ES, CB>), dim3((unsigned)nbx * nby, np), dim3(64 * kStripWaves), 0, st,
                           (const unsigned char*)src + p0 * plane_stride, (unsigned char*)dst + p0 * plane_stride,
                           H, W, pitch, plane_stride, dtype, nbx, aligned);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t mf_strip3_launch_p16(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                                long long pitch, int dtype, hipStream_t st)
{
    return dtype == MF_U8 ? strip3_launch<1, 8>(src, dst, planes, plane_stride, H, W, pitch, dtype, st)
                          : strip3_launch<2, 16>(src, dst, planes, plane_stride, H, W, pitch, dtype, st);
}

hipError_t mf_strip3_launch_u32(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                                long long pitch, int dtype, hipStream_t st)
{
    return strip3_launch<4, 16>(src, dst, planes, plane_stride, H, W, pitch, dtype, st);
}
