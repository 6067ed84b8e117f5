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
// Each wave owns a strip of 64 lanes x P pixels (one 16-byte chunk per lane
// and row) and R = 16 output rows; a lane holds the 18 input rows of its
// chunk in registers, all loaded up front (no LDS, no barriers), so 18
// independent 16-byte loads per lane are in flight. The columns just left and
// right of a lane's chunk come from the neighbouring lanes by a lane shuffle;
// lanes 0 and 63 load theirs. A work-group stacks 4 waves vertically.
#include "mf_internal.h"

namespace {

constexpr int kStripRows = 16;     // output rows per wave
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

template <int ES>
__device__ __forceinline__ uint32_t strip_elem(const uint4& q, int e)
{
    const uint32_t w = e * ES / 4 == 0 ? q.x : e * ES / 4 == 1 ? q.y : e * ES / 4 == 2 ? q.z : q.w;
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

template <int ES>
__global__ void __launch_bounds__(64 * kStripWaves)
mf_strip3_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int H, int W,
                 long long pitch, long long plane_stride, int dtype, int nbx, int aligned)
{
    src += (long long)blockIdx.y * plane_stride;   // plane = blockIdx.y
    dst += (long long)blockIdx.y * plane_stride;
    constexpr int P = 16 / ES;               // pixels per lane
    constexpr int R = kStripRows;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
    const int x0 = bx * 64 * P + lane * P;    // first pixel of this lane's chunk
    const int y0 = (by * kStripWaves + wv) * R;
    if (y0 >= H) return;                      // whole wave; the kernel has no barriers
    const bool key = ES == 4 && dtype == MF_F32;
    const bool whole = aligned && x0 + P <= W; // the 16-byte chunk lies inside the row

    // the chunk of every input row y0-1 .. y0+R (replicate border by clamping)
    // Each branch issues all of its loads before it uses any, so their
    // latencies overlap (a wave at the right edge runs both branches).
    uint4 raw[R + 2];
    uint32_t hv[R + 2];                       // lane 0: pixel x0-1; lane 63: pixel x0+P
    if (whole) {
#pragma unroll
        for (int i = 0; i < R + 2; ++i) {
            const int gy = min(max(y0 - 1 + i, 0), H - 1);
            raw[i] = *(const uint4*)(src + (long long)gy * pitch + (long long)x0 * ES);
        }
    } else if (x0 >= W) {
        // past the right edge: every pixel is column W-1 (replicate border)
#pragma unroll
        for (int i = 0; i < R + 2; ++i) {
            const int gy = min(max(y0 - 1 + i, 0), H - 1);
            uint32_t v = strip_load1<ES>(src + (long long)gy * pitch, W - 1);
            if constexpr (ES == 1) v *= 0x01010101u;
            if constexpr (ES == 2) v *= 0x00010001u;
            raw[i] = make_uint4(v, v, v, v);
        }
    } else {
#pragma unroll
        for (int i = 0; i < R + 2; ++i) {
            const int gy = min(max(y0 - 1 + i, 0), H - 1);
            const unsigned char* row = src + (long long)gy * pitch;
            uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < P; ++e)
                w[e * ES / 4] |= strip_load1<ES>(row, min(x0 + e, W - 1)) << (8 * ((e * ES) % 4));
            raw[i] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
#pragma unroll
    for (int i = 0; i < R + 2; ++i) hv[i] = 0;
    if (lane == 0 || lane == 63) {
        const int hx = lane == 0 ? max(x0 - 1, 0) : min(x0 + P, W - 1);
#pragma unroll
        for (int i = 0; i < R + 2; ++i) {
            const int gy = min(max(y0 - 1 + i, 0), H - 1);
            hv[i] = strip_load1<ES>(src + (long long)gy * pitch, hx);
        }
    }

    // row i as P + 2 keys: [0] = column x0-1, [1..P] = the chunk, [P+1] = x0+P
    auto unpack = [&](int i, uint32_t* v) {
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const uint32_t u = strip_elem<ES>(raw[i], e);
            v[e + 1] = key ? strip_key(u) : u;
        }
        const uint32_t left = __shfl_up(v[P], 1), right = __shfl_down(v[1], 1);
        const uint32_t h = key ? strip_key(hv[i]) : hv[i];
        v[0] = lane == 0 ? h : left;
        v[P + 1] = lane == 63 ? h : right;
    };

    uint32_t a[P + 2], b[P + 2], c[P + 2];
    unpack(0, a);
    unpack(1, b);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        unpack(i + 2, c);
        // sorted columns (initialisation, shared by the three windows)
        uint32_t lo[P + 2], mi[P + 2], hi[P + 2];
#pragma unroll
        for (int e = 0; e < P + 2; ++e) {
            lo[e] = smin(smin(a[e], b[e]), c[e]);
            hi[e] = smax(smax(a[e], b[e]), c[e]);
            mi[e] = smed3(a[e], b[e], c[e]);
        }
        // pruned three-way merge of the window's columns down to the median
        uint32_t o[P];
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const uint32_t l = smax(smax(lo[e], lo[e + 1]), lo[e + 2]);
            const uint32_t m = smed3(mi[e], mi[e + 1], mi[e + 2]);
            const uint32_t h = smin(smin(hi[e], hi[e + 1]), hi[e + 2]);
            o[e] = smed3(l, m, h);
            if (key) o[e] = strip_unkey(o[e]);
        }
        const int y = y0 + i;
        if (y < H) {
            unsigned char* row = dst + (long long)y * pitch;
            if (whole) {
                uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
                for (int e = 0; e < P; ++e) w[e * ES / 4] |= o[e] << (8 * ((e * ES) % 4));
                *(uint4*)(row + (long long)x0 * ES) = make_uint4(w[0], w[1], w[2], w[3]);
            } else {
#pragma unroll
                for (int e = 0; e < P; ++e)
                    if (x0 + e < W) strip_store1<ES>(row, x0 + e, o[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < P + 2; ++e) {
            a[e] = b[e];
            b[e] = c[e];
        }
    }
}

template <int ES>
hipError_t strip3_launch(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                         long long pitch, int dtype, hipStream_t st)
{
    constexpr int span = 64 * (16 / ES);
    const int nbx = (W + span - 1) / span;
    const int nby = (H + kStripRows * kStripWaves - 1) / (kStripRows * kStripWaves);
    // 16-byte chunk loads and stores need 16-byte aligned rows
    const int aligned = ((uintptr_t)src % 16 == 0 && (uintptr_t)dst % 16 == 0 && pitch % 16 == 0 &&
                         plane_stride % 16 == 0) ? 1 : 0;
    for (int p0 = 0; p0 < planes; p0 += 65535) {     // grid rows are planes
        const int np = planes - p0 < 65535 ? planes - p0 : 65535;
        hipLaunchKernelGGL((mf_strip3_kernel<ES>), dim3((unsigned)nbx * nby, np), dim3(64 * kStripWaves), 0, st,
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
    return dtype == MF_U8 ? strip3_launch<1>(src, dst, planes, plane_stride, H, W, pitch, dtype, st)
                          : strip3_launch<2>(src, dst, planes, plane_stride, H, W, pitch, dtype, st);
}

hipError_t mf_strip3_launch_u32(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                                long long pitch, int dtype, hipStream_t st)
{
    return strip3_launch<4>(src, dst, planes, plane_stride, H, W, pitch, dtype, st);
}
