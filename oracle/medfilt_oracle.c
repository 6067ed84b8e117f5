/*
 * Plain CPU oracle for the exact k x k median filter (and its kw x kh
 * rectangular generalisation).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the reference that the GPU path is
 * checked against; it is never part of the product path. It shares no code,
 * header, table or constant with the HIP library.
 *
 * What it computes (Sugy, "A Fast Parallel Median Filtering Algorithm Using
 * Hierarchical Tiling", SIGGRAPH 2025, Section 1): every output pixel is the
 * median of the k x k neighbourhood centred on it. The hierarchical-tiling
 * method returns exactly this value (the 1x1 leaf's sorted core holds the
 * median, Section 3.2), so the oracle is the definition written out:
 *
 *   r = (k-1)/2, N = k*k, m = (N-1)/2
 *   B(i, n) = min(max(i, 0), n-1)                       replicate border
 *   W(y,x)  = { src[B(y+dy,H)][B(x+dx,W)] : dy,dx in [-r, r] }
 *   out(y,x) = element of rank m (0-based) of W(y,x) under the dtype's order
 * A kw x kh window (odd kw columns, odd kh rows) takes dx in [-(kw-1)/2,
 * (kw-1)/2], dy in [-(kh-1)/2, (kh-1)/2], N = kw*kh. The 3-D filter takes a
 * kx x ky x kz box over a volume in the same way, clamping each axis.
 *
 * The paper states no border rule, no float semantics and no gradient; the
 * readings used here are:
 *   - border: replicate (clamp the coordinates);
 *   - float32: IEEE 754 totalOrder on the bit patterns (-NaN < -inf < ... <
 *     -0 < +0 < ... < +inf < +NaN), so equal rank means identical bits;
 *   - argmedian: among the window pixels whose bits equal the median, the one
 *     reached first in row-major (dy outer, dx inner) order, reported as its
 *     plane-flat index B(y+dy)*W + B(x+dx);
 *   - gradient: grad_in = +0, then for p = 0 .. H*W-1 in ascending order
 *     grad_in[idx[p]] += grad_out[p] in binary32.
 *
 * Selection is Hoare's FIND (quickselect) with a three-way partition, so runs
 * of equal values cost linear time. Parity pins: the "not gpu" oracle tests
 * (full-sort brute force, threshold decomposition for 8-bit data, rank
 * certificates, monotone maps, impulses, ramps, float specials, finite
 * differences of the gradient).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_U8 = 0, OR_U16 = 1, OR_U32 = 2, OR_F32 = 3 };

/* Order key: a signed 64-bit integer whose natural order is the dtype's
 * order. For float32 the key is the bit pattern read as int32 with the low
 * 31 bits flipped when the sign bit is set (IEEE totalOrder). The map is an
 * involution on the 32-bit pattern, so key_to_bits undoes it. */
static int64_t f32_bits_to_key(uint32_t bits)
{
    int32_t i = (int32_t)bits;
    if (i < 0)
        i = (int32_t)(bits ^ 0x7FFFFFFFu);
    return (int64_t)i;
}

static uint32_t f32_key_to_bits(int64_t key)
{
    uint32_t u = (uint32_t)(int32_t)key;
    if ((int32_t)u < 0)
        u ^= 0x7FFFFFFFu;
    return u;
}

static int64_t load_key(const unsigned char* base, int64_t pitch_bytes, int dtype,
                        int64_t y, int64_t x)
{
    const unsigned char* row = base + y * pitch_bytes;
    switch (dtype) {
    case OR_U8:  return (int64_t)((const uint8_t*)row)[x];
    case OR_U16: return (int64_t)((const uint16_t*)row)[x];
    case OR_U32: return (int64_t)((const uint32_t*)row)[x];
    default: {
        uint32_t b;
        memcpy(&b, row + 4 * x, 4);
        return f32_bits_to_key(b);
    }
    }
}

static void store_key(unsigned char* base, int64_t pitch_bytes, int dtype,
                      int64_t y, int64_t x, int64_t key)
{
    unsigned char* row = base + y * pitch_bytes;
    switch (dtype) {
    case OR_U8:  ((uint8_t*)row)[x] = (uint8_t)key; break;
    case OR_U16: ((uint16_t*)row)[x] = (uint16_t)key; break;
    case OR_U32: ((uint32_t*)row)[x] = (uint32_t)key; break;
    default: {
        uint32_t b = f32_key_to_bits(key);
        memcpy(row + 4 * x, &b, 4);
    }
    }
}

static int64_t clamp_index(int64_t i, int64_t n)
{
    if (i < 0) return 0;
    if (i > n - 1) return n - 1;
    return i;
}

/* Rank-`rank` element (0-based) of a[0..n), which is permuted in place.
 * Hoare's FIND: partition around a pivot into < / == / > and keep only the
 * part that holds the wanted rank. */
static int64_t select_rank(int64_t* a, int64_t n, int64_t rank)
{
    int64_t lo = 0, hi = n; /* the wanted element lies in a[lo..hi) */
    for (;;) {
        if (hi - lo == 1)
            return a[lo];
        /* median-of-three pivot value */
        int64_t p0 = a[lo], p1 = a[lo + (hi - lo) / 2], p2 = a[hi - 1];
        int64_t pivot;
        if ((p0 <= p1 && p1 <= p2) || (p2 <= p1 && p1 <= p0)) pivot = p1;
        else if ((p1 <= p0 && p0 <= p2) || (p2 <= p0 && p0 <= p1)) pivot = p0;
        else pivot = p2;
        /* three-way partition: a[lo..lt) < pivot, a[lt..i) == pivot,
         * a[gt..hi) > pivot */
        int64_t lt = lo, i = lo, gt = hi;
        while (i < gt) {
            if (a[i] < pivot) {
                int64_t t = a[i]; a[i] = a[lt]; a[lt] = t;
                ++lt; ++i;
            } else if (a[i] > pivot) {
                --gt;
                int64_t t = a[i]; a[i] = a[gt]; a[gt] = t;
            } else {
                ++i;
            }
        }
        if (rank < lt) hi = lt;
        else if (rank < gt) return pivot;
        else lo = gt;
    }
}

static int check_args(const void* src, const void* dst, int64_t H, int64_t W,
                      int64_t pitch_bytes, int dtype, int kw, int kh)
{
    static const int size_of[4] = {1, 2, 4, 4};
    if (!src || !dst) return -1;
    if (H < 1 || W < 1) return -2;
    if (dtype < 0 || dtype > 3) return -4;
    if (pitch_bytes < W * size_of[dtype] || pitch_bytes % size_of[dtype]) return -3;
    if (kw < 1 || (kw % 2) == 0 || kh < 1 || (kh % 2) == 0) return -5;
    return 0;
}

/* Median of the kw x kh window (kw columns, kh rows) around (y, x): fills
 * `buf` (kw*kh entries) in row-major window order and selects rank
 * (kw*kh - 1) / 2. */
static int64_t window_median(const unsigned char* src, int64_t H, int64_t W,
                             int64_t pitch_bytes, int dtype, int kw, int kh,
                             int64_t y, int64_t x, int64_t* buf)
{
    const int rx = (kw - 1) / 2, ry = (kh - 1) / 2;
    int64_t n = 0;
    for (int dy = -ry; dy <= ry; ++dy) {
        const int64_t yy = clamp_index(y + dy, H);
        for (int dx = -rx; dx <= rx; ++dx)
            buf[n++] = load_key(src, pitch_bytes, dtype, yy, clamp_index(x + dx, W));
    }
    return select_rank(buf, n, (n - 1) / 2);
}

/* Median filter with a kw x kh window (odd sides; kw along rows, kh along
 * columns) of rows [row_begin, row_end) of an H x W plane. src and dst share
 * pitch_bytes. Returns 0, or a negative code on a bad argument. */
int oracle_median_filter_rect(const void* src, void* dst, int64_t H, int64_t W,
                              int64_t pitch_bytes, int dtype, int kw, int kh,
                              int64_t row_begin, int64_t row_end, int nthreads)
{
    int rc = check_args(src, dst, H, W, pitch_bytes, dtype, kw, kh);
    if (rc) return rc;
    if (row_begin < 0) row_begin = 0;
    if (row_end > H) row_end = H;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int64_t N = (int64_t)kw * kh;
#pragma omp parallel
    {
        int64_t* buf = (int64_t*)malloc((size_t)N * sizeof(int64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t y = row_begin; y < row_end; ++y)
            for (int64_t x = 0; x < W; ++x)
                store_key((unsigned char*)dst, pitch_bytes, dtype, y, x,
                          window_median((const unsigned char*)src, H, W, pitch_bytes,
                                        dtype, kw, kh, y, x, buf));
        free(buf);
    }
    return 0;
}

/* The k x k filter (Section 1). */
int oracle_median_filter(const void* src, void* dst, int64_t H, int64_t W,
                         int64_t pitch_bytes, int dtype, int k,
                         int64_t row_begin, int64_t row_end, int nthreads)
{
    return oracle_median_filter_rect(src, dst, H, W, pitch_bytes, dtype, k, k, row_begin, row_end,
                                     nthreads);
}

/* Median of the kw x kh window at n individual pixels (ys[i], xs[i]); out is
 * a dense array of n elements of the dtype. */
int oracle_median_points_rect(const void* src, int64_t H, int64_t W, int64_t pitch_bytes,
                              int dtype, int kw, int kh, const int64_t* ys, const int64_t* xs,
                              int64_t n, void* out, int nthreads)
{
    int rc = check_args(src, out, H, W, pitch_bytes, dtype, kw, kh);
    if (rc) return rc;
    if (!ys || !xs) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int64_t N = (int64_t)kw * kh;
    static const int size_of[4] = {1, 2, 4, 4};
    const int64_t out_pitch = n * size_of[dtype];
#pragma omp parallel
    {
        int64_t* buf = (int64_t*)malloc((size_t)N * sizeof(int64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t y = ys[i], x = xs[i];
            if (y < 0 || y >= H || x < 0 || x >= W) continue;
            store_key((unsigned char*)out, out_pitch, dtype, 0, i,
                      window_median((const unsigned char*)src, H, W, pitch_bytes,
                                    dtype, kw, kh, y, x, buf));
        }
        free(buf);
    }
    return 0;
}

int oracle_median_points(const void* src, int64_t H, int64_t W, int64_t pitch_bytes,
                         int dtype, int k, const int64_t* ys, const int64_t* xs,
                         int64_t n, void* out, int nthreads)
{
    return oracle_median_points_rect(src, H, W, pitch_bytes, dtype, k, k, ys, xs, n, out, nthreads);
}

/* 3-D median filter (the paper's future-work extension to volumes, Section
 * 7.2): every output voxel is the median of the kx x ky x kz box centred on
 * it, coordinates clamped in each axis (replicate border), rank
 * (kx*ky*kz - 1) / 2. The volume is D slices of H rows of W elements; rows
 * are pitch_bytes apart and slices slice_bytes apart (src and dst share
 * both). Slices [z_begin, z_end) are computed. Returns 0 or a negative code
 * on a bad argument. */
int oracle_median_filter_3d(const void* src, void* dst, int64_t D, int64_t H, int64_t W,
                            int64_t pitch_bytes, int64_t slice_bytes, int dtype, int kx, int ky,
                            int kz, int64_t z_begin, int64_t z_end, int nthreads)
{
    static const int size_of[4] = {1, 2, 4, 4};
    int rc = check_args(src, dst, H, W, pitch_bytes, dtype, kx, ky);
    if (rc) return rc;
    if (D < 1) return -2;
    if (kz < 1 || (kz % 2) == 0) return -5;
    if (slice_bytes < (H - 1) * pitch_bytes + W * size_of[dtype] || slice_bytes % size_of[dtype]) return -3;
    if (z_begin < 0) z_begin = 0;
    if (z_end > D) z_end = D;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int rx = (kx - 1) / 2, ry = (ky - 1) / 2, rz = (kz - 1) / 2;
    const int64_t N = (int64_t)kx * ky * kz;
    const unsigned char* s8 = (const unsigned char*)src;
    unsigned char* d8 = (unsigned char*)dst;
#pragma omp parallel
    {
        int64_t* buf = (int64_t*)malloc((size_t)N * sizeof(int64_t));
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int64_t z = z_begin; z < z_end; ++z)
            for (int64_t y = 0; y < H; ++y)
                for (int64_t x = 0; x < W; ++x) {
                    int64_t n = 0;
                    for (int dz = -rz; dz <= rz; ++dz) {
                        const unsigned char* sl = s8 + clamp_index(z + dz, D) * slice_bytes;
                        for (int dy = -ry; dy <= ry; ++dy) {
                            const int64_t yy = clamp_index(y + dy, H);
                            for (int dx = -rx; dx <= rx; ++dx)
                                buf[n++] = load_key(sl, pitch_bytes, dtype, yy, clamp_index(x + dx, W));
                        }
                    }
                    store_key(d8 + z * slice_bytes, pitch_bytes, dtype, y, x, select_rank(buf, n, (n - 1) / 2));
                }
        free(buf);
    }
    return 0;
}

/* Median value and argmedian of rows [row_begin, row_end) of a contiguous
 * float32 plane. idx is the plane-flat index of the first window pixel, in
 * row-major window order, whose bits equal the median. */
int oracle_argmedian_f32(const float* src, float* val, int32_t* idx, int64_t H, int64_t W,
                         int k, int64_t row_begin, int64_t row_end, int nthreads)
{
    int rc = check_args(src, val, H, W, W * 4, OR_F32, k, k);
    if (rc) return rc;
    if (!idx) return -1;
    if (row_begin < 0) row_begin = 0;
    if (row_end > H) row_end = H;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int r = (k - 1) / 2;
    const int64_t N = (int64_t)k * k;
#pragma omp parallel
    {
        int64_t* buf = (int64_t*)malloc((size_t)N * sizeof(int64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t y = row_begin; y < row_end; ++y)
            for (int64_t x = 0; x < W; ++x) {
                int64_t key = window_median((const unsigned char*)src, H, W, W * 4,
                                            OR_F32, k, k, y, x, buf);
                uint32_t bits = f32_key_to_bits(key);
                int64_t found = -1;
                for (int dy = -r; dy <= r && found < 0; ++dy) {
                    const int64_t yy = clamp_index(y + dy, H);
                    for (int dx = -r; dx <= r; ++dx) {
                        const int64_t xx = clamp_index(x + dx, W);
                        uint32_t b;
                        memcpy(&b, &src[yy * W + xx], 4);
                        if (b == bits) { found = yy * W + xx; break; }
                    }
                }
                memcpy(&val[y * W + x], &bits, 4);
                idx[y * W + x] = (int32_t)found;
            }
        free(buf);
    }
    return 0;
}

/* Gradient of a median filter with respect to its input, for one float32
 * plane of n pixels: scatter of grad_out through idx in ascending output
 * order, binary32 additions starting from +0. */
int oracle_grad_f32(const float* grad_out, const int32_t* idx, float* grad_in, int64_t n)
{
    if (!grad_out || !idx || !grad_in) return -1;
    for (int64_t q = 0; q < n; ++q)
        grad_in[q] = 0.0f;
    for (int64_t p = 0; p < n; ++p) {
        int32_t q = idx[p];
        if (q < 0 || q >= n) return -2;
        volatile float s = grad_in[q] + grad_out[p]; /* one rounded add, no contraction */
        grad_in[q] = s;
    }
    return 0;
}
