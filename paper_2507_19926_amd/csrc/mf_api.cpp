// C ABI of the median filter: argument validation, configuration choice and
// dispatch to the compiled kernels. Every check runs on the host before any
// GPU call, so a bad argument never reaches a kernel.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "mf_internal.h"

#define MF_OBL_ENTRY(NET, K, TW, TH, RY, NW, INL) MF_OBL_DECLARE(NET, RY, NW)
#include "mf_obl_table.inc"
#undef MF_OBL_ENTRY
#define MF_OBL_RECT_ENTRY(NET, KW, KH, TW, TH, RY, NW, INL) MF_OBL_DECLARE(NET, RY, NW)
#include "mf_obl_rect_table.inc"
#undef MF_OBL_RECT_ENTRY

namespace {

// form: 1 = column segments sorted once per work-group and shared, 2 = each
// tile sorts its own columns, 3 = column-strip streaming form (k = 3, no
// batched kernel of its own).
struct OblEntry {
    int k, tw, th, ry, nw, form;
    mf_launch_fn p16, u32;
    void (*batched_p16)(MfBatchedKernel*);
    void (*batched_u32)(MfBatchedKernel*);
};

const OblEntry kOblTable[] = {
#define MF_OBL_ENTRY(NET, K, TW, TH, RY, NW, INL)                                                    \
    {K, TW, TH, RY, NW, (INL) ? 2 : 1, MF_OBL_NAME(NET, RY, NW, p16), MF_OBL_NAME(NET, RY, NW, u32), \
     MF_OBL_BATCHED_NAME(NET, RY, NW, p16), MF_OBL_BATCHED_NAME(NET, RY, NW, u32)},
#include "mf_obl_table.inc"
#undef MF_OBL_ENTRY
    {3, 1, 1, 16, 4, 3, mf_strip3_launch_p16, mf_strip3_launch_u32, nullptr, nullptr},
};
constexpr int kOblCount = sizeof(kOblTable) / sizeof(kOblTable[0]);

// Oblivious networks for rectangular windows (k_w columns by k_h rows).
struct OblRectEntry {
    int kw, kh, tw, th;
    mf_launch_fn p16, u32;
};

const OblRectEntry kOblRectTable[] = {
#define MF_OBL_RECT_ENTRY(NET, KW, KH, TW, TH, RY, NW, INL) \
    {KW, KH, TW, TH, MF_OBL_NAME(NET, RY, NW, p16), MF_OBL_NAME(NET, RY, NW, u32)},
#include "mf_obl_rect_table.inc"
#undef MF_OBL_RECT_ENTRY
    {0, 0, 0, 0, nullptr, nullptr},   // keeps the array non-empty
};

const OblRectEntry* find_obl_rect(int kw, int kh)
{
    for (const OblRectEntry& e : kOblRectTable)
        if (e.p16 && e.kw == kw && e.kh == kh) return &e;
    return nullptr;
}

constexpr int kMaxK = 75;

// Measured AUTO choices (class 0: 8-bit data, and 16-bit data without a
// class 2 entry; class 1: 32-bit data; class 2: 16-bit data). 8- and 16-bit
// data share the oblivious networks, but the data-aware kernel holds 8-bit
// data in bytes and 16-bit data in 16-bit elements, so their best tiles
// differ.
struct AutoEntry {
    int cls, k, variant, tw, th, group, form, rows;
};
const AutoEntry kAutoTable[] = {
#define MF_AUTO(C, K, V, TW, TH, G, F, R) {C, K, V, TW, TH, G, F, R},
#include "mf_auto_table.inc"
#undef MF_AUTO
    {-1, 0, 0, 0, 0, 0, 0, 0}};

thread_local std::string g_last_error;

int32_t fail(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t fail(int32_t code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int elem_size(int32_t dtype)
{
    switch (dtype) {
    case MF_U8: return 1;
    case MF_U16: return 2;
    case MF_U32: return 4;
    case MF_F32: return 4;
    default: return 0;
    }
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// The column-strip form is only returned when asked for (form 3).
const OblEntry* find_obl(int k, int tw, int th, int nw, int form, int rows)
{
    for (int i = 0; i < kOblCount; ++i) {
        const OblEntry& e = kOblTable[i];
        if (e.k == k && (tw == 0 || e.tw == tw) && (th == 0 || e.th == th) && (nw == 0 || e.nw == nw) &&
            (form == 0 ? e.form != 3 : e.form == form) && (rows == 0 || e.ry == rows))
            return &e;  // the table lists each k's preferred configuration first
    }
    return nullptr;
}

// Resolve (dtype, k, opt) to a variant and root tile. Host only.
int32_t resolve(int32_t dtype, int32_t k, const mf_options* opt, int32_t* variant, int32_t* tw,
                int32_t* th, const OblEntry** obl, int32_t* group = nullptr, int32_t* da_form = nullptr)
{
    mf_options o = {};
    if (opt) o = *opt;
    if (o.variant < MF_VARIANT_AUTO || o.variant > MF_VARIANT_DATA_AWARE)
        return fail(MF_ERR_CONFIG, "unknown variant %d", o.variant);
    if (o.group != 0 && o.group != 1 && o.group != 2 && o.group != 4)
        return fail(MF_ERR_CONFIG, "tiles per work-group %d not in {0, 1, 2, 4}", o.group);
    if (group) *group = 0;
    if (da_form) *da_form = 0;
    if ((o.tile_w && (!pow2(o.tile_w) || o.tile_w > k)) || (o.tile_h && (!pow2(o.tile_h) || o.tile_h > k)) ||
        o.tile_w < 0 || o.tile_h < 0)
        return fail(MF_ERR_CONFIG, "root tile %dx%d is not a pair of powers of two <= k=%d", o.tile_w,
                    o.tile_h, k);
    if (o.form < 0 || o.form > 3) return fail(MF_ERR_CONFIG, "form %d not in {0, 1, 2, 3}", o.form);
    *obl = nullptr;
    // measured choice for this (value class, k), when nothing was requested
    if (o.rows < 0) return fail(MF_ERR_CONFIG, "rows %d must be >= 0", o.rows);
    if (o.variant == MF_VARIANT_AUTO && !o.tile_w && !o.tile_h && !o.group && !o.form && !o.rows) {
        int cls = (dtype == MF_U8 || dtype == MF_U16) ? 0 : 1;
        if (dtype == MF_U16)
            for (const AutoEntry& a : kAutoTable)
                if (a.cls == 2 && a.k == k) cls = 2;
        for (const AutoEntry& a : kAutoTable) {
            if (a.cls != cls || a.k != k) continue;
            if (a.variant == MF_VARIANT_OBLIVIOUS) {
                const OblEntry* e = find_obl(k, a.tw, a.th, a.group, a.form, a.rows);
                if (e) {
                    *variant = MF_VARIANT_OBLIVIOUS;
                    *tw = e->tw;
                    *th = e->th;
                    *obl = e;
                    return MF_OK;
                }
            } else if (mf_da_supports(dtype, k, a.tw, a.th, a.group, 0, a.form)) {
                *variant = MF_VARIANT_DATA_AWARE;
                *tw = a.tw;
                *th = a.th;
                if (group) *group = a.group;
                if (da_form) *da_form = a.form;
                return MF_OK;
            }
            break;  // a stale entry: fall back to the built-in order
        }
    }
    if (o.variant != MF_VARIANT_DATA_AWARE) {
        const OblEntry* e =
            find_obl(k, o.tile_w, o.tile_h, o.group == 1 || o.group == 4 ? o.group : 0, o.form, o.rows);
        if (e) {
            *variant = MF_VARIANT_OBLIVIOUS;
            *tw = e->tw;
            *th = e->th;
            *obl = e;
            return MF_OK;
        }
        if (o.variant == MF_VARIANT_OBLIVIOUS)
            return fail(MF_ERR_CONFIG, "no oblivious network compiled for k=%d tile %dx%d", k, o.tile_w,
                        o.tile_h);
    }
    // data-aware: form 1 = rounds per recursion level, 2 = rounds over the
    // whole schedule (3 is the oblivious column-strip form only)
    int dtw = o.tile_w, dth = o.tile_h, dg = o.group, df = o.form;
    if (df == 3) return fail(MF_ERR_CONFIG, "form 3 is the oblivious column-strip form (k = 3)");
    if (!dtw && !dth && !dg && !df) {
        mf_da_default_tile(dtype, k, &dtw, &dth, &dg, 0, &df);
    }
    if (!mf_da_supports(dtype, k, dtw, dth, dg, 0, df))
        return fail(MF_ERR_CONFIG, "data-aware variant does not support k=%d tile %dx%d group %d form %d", k, dtw,
                    dth, dg, df);
    *variant = MF_VARIANT_DATA_AWARE;
    *tw = dtw;
    *th = dth;
    if (group) *group = dg;
    if (da_form) *da_form = df;
    return MF_OK;
}

int32_t validate(const void* src, const void* dst, int64_t H, int64_t W, int64_t pitch, int32_t dtype,
                 int32_t k, int32_t border)
{
    if (!src || !dst) return fail(MF_ERR_NULL, "src or dst is NULL");
    const int s = elem_size(dtype);
    if (!s) return fail(MF_ERR_DTYPE, "unknown dtype %d", dtype);
    if (H < 1 || W < 1 || H > (1 << 30) || W > (1 << 30))
        return fail(MF_ERR_DIMS, "H=%lld W=%lld outside [1, 2^30]", (long long)H, (long long)W);
    if (pitch < W * s || pitch % s || pitch > ((int64_t)1 << 40))
        return fail(MF_ERR_PITCH, "pitch %lld invalid for W=%lld of %d-byte elements", (long long)pitch,
                    (long long)W, s);
    if (((uintptr_t)src | (uintptr_t)dst) % s)
        return fail(MF_ERR_PITCH, "src/dst not aligned to the %d-byte element size", s);
    if (k < 1 || k % 2 == 0 || k > kMaxK) return fail(MF_ERR_K, "k=%d must be odd in [1, %d]", k, kMaxK);
    if (border != MF_BORDER_REPLICATE) return fail(MF_ERR_BORDER, "unknown border mode %d", border);
    const uintptr_t a0 = (uintptr_t)src, b0 = (uintptr_t)dst;
    const uintptr_t len = (uintptr_t)((H - 1) * pitch + W * s);
    if (a0 < b0 + len && b0 < a0 + len) return fail(MF_ERR_ALIAS, "src and dst overlap");
    return MF_OK;
}

int32_t hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return MF_OK;
    return fail(MF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

int32_t mf_internal_validate(const void* src, const void* dst, int64_t H, int64_t W, int64_t pitch,
                             int32_t dtype, int32_t k, int32_t border)
{
    return validate(src, dst, H, W, pitch, dtype, k, border);
}

int32_t mf_internal_fail(int32_t code, const char* msg) { return fail(code, "%s", msg); }

int32_t mf_internal_resolve(int32_t dtype, int32_t k, int32_t* variant, int32_t* tw, int32_t* th,
                            int32_t* group, MfBatchedKernel* obl_p16, MfBatchedKernel* obl_u32, int32_t* da_form)
{
    const OblEntry* e = nullptr;
    int32_t rc = resolve(dtype, k, nullptr, variant, tw, th, &e, group, da_form);
    if (rc) return rc;
    // the column-strip form has no batched kernel: plans use k's default
    // network
    if (e && e->form == 3) e = find_obl(k, 0, 0, 0, 0, 0);
    if (e) {
        e->batched_p16(obl_p16);
        e->batched_u32(obl_u32);
    }
    return MF_OK;
}

// Plane count and stride of a multi-plane call (src, dst and the single-plane
// arguments already validated). planes = 1 sets the stride to 0.
static int32_t check_planes(const void* src, const void* dst, int64_t planes, int64_t* plane_stride_bytes,
                            int64_t H, int64_t W, int64_t pitch_bytes, int32_t dtype)
{
    const int s = elem_size(dtype);
    const int64_t plane_bytes = (H - 1) * pitch_bytes + W * s;
    if (planes < 1 || planes > ((int64_t)1 << 30))
        return fail(MF_ERR_DIMS, "planes=%lld outside [1, 2^30]", (long long)planes);
    if (planes > 1) {
        const int64_t ps = *plane_stride_bytes;
        if (ps < plane_bytes || ps % s || ps > ((int64_t)1 << 46))
            return fail(MF_ERR_PITCH, "plane stride %lld: planes of %lld bytes would overlap or misalign",
                        (long long)ps, (long long)plane_bytes);
        const uintptr_t a0 = (uintptr_t)src, b0 = (uintptr_t)dst;
        const uintptr_t len = (uintptr_t)((planes - 1) * ps + plane_bytes);
        if (a0 < b0 + len && b0 < a0 + len) return fail(MF_ERR_ALIAS, "src and dst plane ranges overlap");
    } else {
        *plane_stride_bytes = 0;
    }
    return MF_OK;
}

// Global-memory form through median_filter_ex / median_filter_planes: the
// workspace (all tiles at once, capped at kGlobalBudget; larger images run
// in slices) is allocated and freed in stream order around the launches.
constexpr long long kGlobalBudget = 256LL << 20;

static int32_t global_tile_option(int32_t k, const mf_options* opt, int32_t* tw, int32_t* th)
{
    *tw = opt ? opt->tile_w : 0;
    *th = opt ? opt->tile_h : 0;
    if (opt && (opt->group || opt->form || opt->rows))
        return fail(MF_ERR_CONFIG, "the global-memory form takes only a root tile");
    if ((*tw && (!pow2(*tw) || *tw > k)) || (*th && (!pow2(*th) || *th > k)) || *tw < 0 || *th < 0 ||
        ((*tw == 0) != (*th == 0)))
        return fail(MF_ERR_CONFIG, "root tile %dx%d is not a pair of powers of two <= k=%d (or 0x0)", *tw, *th, k);
    return MF_OK;
}

static int32_t global_with_own_workspace(const void* src, void* dst, int64_t planes, int64_t plane_stride,
                                         int64_t H, int64_t W, int64_t pitch, int32_t dtype, int32_t k,
                                         const mf_options* opt, hipStream_t st)
{
    int32_t tw = 0, th = 0;
    int32_t rc = global_tile_option(k, opt, &tw, &th);
    if (rc) return rc;
    long long slot = 0, all = 0;
    int utw = 0, uth = 0;
    if (!mf_dag_workspace(dtype, k, tw, th, planes, (int)H, (int)W, &slot, &all, &utw, &uth))
        return fail(MF_ERR_CONFIG, "no global-memory schedule for k=%d tile %dx%d", k, tw, th);
    long long bytes = all < kGlobalBudget ? all : kGlobalBudget;
    if (bytes < slot) bytes = slot;
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, (size_t)bytes, st);
    if (e != hipSuccess) return fail(MF_ERR_NOMEM, "workspace of %lld bytes: %s", bytes, hipGetErrorString(e));
    e = mf_dag_launch(src, dst, (int)planes, plane_stride, (int)H, (int)W, pitch, dtype, k, tw, th, ws, bytes, st);
    hipError_t f = hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_status(e, "global-memory kernel launch");
    return hip_status(f, "hipFreeAsync(workspace)");
}

extern "C" {

int32_t median_filter_rect(const void* src, void* dst, int64_t planes, int64_t plane_stride_bytes, int64_t H,
                           int64_t W, int64_t pitch_bytes, int32_t dtype, int32_t kw, int32_t kh, int32_t border,
                           const mf_options* opt, void* stream)
{
    g_last_error.clear();
    const int32_t variant = opt ? opt->variant : MF_VARIANT_AUTO;
    if (kw == kh) {
        mf_options o = {};
        o.variant = variant;
        return median_filter_planes(src, dst, planes, plane_stride_bytes, H, W, pitch_bytes, dtype, kw, border, &o,
                                    stream);
    }
    if (opt && (opt->tile_w || opt->tile_h || opt->group || opt->form || opt->rows))
        return fail(MF_ERR_CONFIG, "a rectangular window takes only the variant option");
    if (variant != MF_VARIANT_AUTO && variant != MF_VARIANT_OBLIVIOUS && variant != MF_VARIANT_DATA_AWARE)
        return fail(MF_ERR_CONFIG, "unknown variant %d", variant);
    // k = 1 stands for the window in the shared checks (it passes the k test)
    int32_t rc = validate(src, dst, H, W, pitch_bytes, dtype, 1, border);
    if (rc) return rc;
    const int side = mf_da_rect_max_side();
    if (kw < 1 || kh < 1 || kw % 2 == 0 || kh % 2 == 0 || kw > side || kh > side)
        return fail(MF_ERR_K, "window %dx%d: a rectangular window needs odd sides in [1, %d]", kw, kh, side);
    rc = check_planes(src, dst, planes, &plane_stride_bytes, H, W, pitch_bytes, dtype);
    if (rc) return rc;
    const OblRectEntry* oe = variant == MF_VARIANT_DATA_AWARE ? nullptr : find_obl_rect(kw, kh);
    if (oe) {
        mf_launch_fn fn = (dtype == MF_U8 || dtype == MF_U16) ? oe->p16 : oe->u32;
        return hip_status(fn(src, dst, (int)planes, plane_stride_bytes, (int)H, (int)W, pitch_bytes, dtype,
                             (hipStream_t)stream),
                          "oblivious kernel launch");
    }
    if (variant == MF_VARIANT_OBLIVIOUS)
        return fail(MF_ERR_CONFIG, "no oblivious network compiled for the %dx%d window", kw, kh);
    if (!mf_da_supports(dtype, kw, 0, 0, 0, kh))
        return fail(MF_ERR_CONFIG, "no data-aware schedule for the %dx%d window", kw, kh);
    return hip_status(mf_da_launch(src, dst, (int)planes, plane_stride_bytes, (int)H, (int)W, pitch_bytes, dtype, kw,
                                   0, 0, 0, (hipStream_t)stream, kh),
                      "data-aware kernel launch");
}

int32_t mf_max_rect_side(void) { return mf_da_rect_max_side(); }

int32_t mf_query_rect_config(int32_t dtype, int32_t kw, int32_t kh, int32_t* variant, int32_t* tile_w,
                             int32_t* tile_h)
{
    g_last_error.clear();
    if (kw == kh) return mf_query_config(dtype, kw, nullptr, variant, tile_w, tile_h);
    if (!variant || !tile_w || !tile_h) return fail(MF_ERR_NULL, "output pointer is NULL");
    if (!elem_size(dtype)) return fail(MF_ERR_DTYPE, "unknown dtype %d", dtype);
    const int side = mf_da_rect_max_side();
    if (kw < 1 || kh < 1 || kw % 2 == 0 || kh % 2 == 0 || kw > side || kh > side)
        return fail(MF_ERR_K, "window %dx%d: a rectangular window needs odd sides in [1, %d]", kw, kh, side);
    if (const OblRectEntry* oe = find_obl_rect(kw, kh)) {
        *variant = MF_VARIANT_OBLIVIOUS;
        *tile_w = oe->tw;
        *tile_h = oe->th;
        return MF_OK;
    }
    int tw = 0, th = 0, g = 0;
    mf_da_default_tile(dtype, kw, &tw, &th, &g, kh);
    if (!tw) return fail(MF_ERR_CONFIG, "no data-aware schedule for the %dx%d window", kw, kh);
    *variant = MF_VARIANT_DATA_AWARE;
    *tile_w = tw;
    *tile_h = th;
    return MF_OK;
}

int32_t median_filter_planes(const void* src, void* dst, int64_t planes, int64_t plane_stride_bytes, int64_t H,
                             int64_t W, int64_t pitch_bytes, int32_t dtype, int32_t k, int32_t border,
                             const mf_options* opt, void* stream)
{
    g_last_error.clear();
    int32_t rc = validate(src, dst, H, W, pitch_bytes, dtype, k, border);
    if (rc) return rc;
    rc = check_planes(src, dst, planes, &plane_stride_bytes, H, W, pitch_bytes, dtype);
    if (rc) return rc;
    const int s = elem_size(dtype);
    hipStream_t st = (hipStream_t)stream;
    if (k == 1) {
        for (int64_t p = 0; p < planes; ++p) {
            rc = hip_status(hipMemcpy2DAsync((char*)dst + p * plane_stride_bytes, pitch_bytes,
                                             (const char*)src + p * plane_stride_bytes, pitch_bytes, W * s, H,
                                             hipMemcpyDeviceToDevice, st),
                            "hipMemcpy2DAsync");
            if (rc) return rc;
        }
        return MF_OK;
    }
    if (opt && opt->variant == MF_VARIANT_GLOBAL)
        return global_with_own_workspace(src, dst, planes, plane_stride_bytes, H, W, pitch_bytes, dtype, k, opt,
                                         st);
    int32_t variant = 0, tw = 0, th = 0, group = 0, da_form = 0;
    const OblEntry* e = nullptr;
    rc = resolve(dtype, k, opt, &variant, &tw, &th, &e, &group, &da_form);
    if (rc) return rc;
    if (variant == MF_VARIANT_OBLIVIOUS) {
        mf_launch_fn fn = (dtype == MF_U8 || dtype == MF_U16) ? e->p16 : e->u32;
        return hip_status(fn(src, dst, (int)planes, plane_stride_bytes, (int)H, (int)W, pitch_bytes, dtype, st),
                          "oblivious kernel launch");
    }
    return hip_status(mf_da_launch(src, dst, (int)planes, plane_stride_bytes, (int)H, (int)W, pitch_bytes, dtype, k,
                                   tw, th, group, st, 0, da_form),
                      "data-aware kernel launch");
}

int32_t median_filter_ex(const void* src, void* dst, int64_t H, int64_t W, int64_t pitch_bytes,
                         int32_t dtype, int32_t k, int32_t border, const mf_options* opt, void* stream)
{
    return median_filter_planes(src, dst, 1, 0, H, W, pitch_bytes, dtype, k, border, opt, stream);
}

int32_t median_filter(const void* src, void* dst, int64_t H, int64_t W, int64_t pitch_bytes,
                      int32_t dtype, int32_t k, int32_t border, void* stream)
{
    return median_filter_ex(src, dst, H, W, pitch_bytes, dtype, k, border, nullptr, stream);
}

int32_t mf_query_config(int32_t dtype, int32_t k, const mf_options* opt, int32_t* variant,
                        int32_t* tile_w, int32_t* tile_h)
{
    g_last_error.clear();
    if (!variant || !tile_w || !tile_h) return fail(MF_ERR_NULL, "output pointer is NULL");
    if (!elem_size(dtype)) return fail(MF_ERR_DTYPE, "unknown dtype %d", dtype);
    if (k < 1 || k % 2 == 0 || k > kMaxK) return fail(MF_ERR_K, "k=%d must be odd in [1, %d]", k, kMaxK);
    if (k == 1) {
        *variant = MF_VARIANT_AUTO;
        *tile_w = *tile_h = 1;
        return MF_OK;
    }
    if (opt && opt->variant == MF_VARIANT_GLOBAL) {
        int64_t slot = 0, all = 0;
        mf_options r = {};
        const int32_t rc = mf_global_workspace(dtype, k, opt->tile_w, opt->tile_h, 1, 1, 1, &slot, &all, &r);
        if (rc) return rc;
        *variant = r.variant;
        *tile_w = r.tile_w;
        *tile_h = r.tile_h;
        return MF_OK;
    }
    const OblEntry* e = nullptr;
    return resolve(dtype, k, opt, variant, tile_w, tile_h, &e);
}

int32_t mf_query_options(int32_t dtype, int32_t k, const mf_options* opt, mf_options* resolved)
{
    g_last_error.clear();
    if (!resolved) return fail(MF_ERR_NULL, "output pointer is NULL");
    if (!elem_size(dtype)) return fail(MF_ERR_DTYPE, "unknown dtype %d", dtype);
    if (k < 1 || k % 2 == 0 || k > kMaxK) return fail(MF_ERR_K, "k=%d must be odd in [1, %d]", k, kMaxK);
    if (opt && opt->variant == MF_VARIANT_GLOBAL && k >= 3) {
        int64_t slot = 0, all = 0;
        return mf_global_workspace(dtype, k, opt->tile_w, opt->tile_h, 1, 1, 1, &slot, &all, resolved);
    }
    mf_options r = {};
    if (k == 1) {
        r.tile_w = r.tile_h = 1;
        *resolved = r;
        return MF_OK;
    }
    const OblEntry* e = nullptr;
    int32_t group = 0, da_form = 0;
    const int32_t rc = resolve(dtype, k, opt, &r.variant, &r.tile_w, &r.tile_h, &e, &group, &da_form);
    if (rc) return rc;
    if (e) {
        r.group = e->nw;
        r.form = e->form;
        r.rows = e->ry;
    } else {
        int tw = 0, th = 0, g = 0, f = 0;
        if (!group || !da_form) mf_da_default_tile(dtype, k, &tw, &th, &g, 0, &f);
        r.group = group ? group : g;
        r.form = da_form ? da_form : f;
    }
    *resolved = r;
    return MF_OK;
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

static int32_t validate_planes(int64_t planes, int64_t H, int64_t W, int32_t k, int32_t border)
{
    if (planes < 1 || H < 1 || W < 1 || H * W >= ((int64_t)1 << 31) || planes > ((int64_t)1 << 31) / 1)
        return fail(MF_ERR_DIMS, "planes=%lld H=%lld W=%lld: need >= 1 and H*W < 2^31", (long long)planes,
                    (long long)H, (long long)W);
    if (k < 1 || k % 2 == 0 || k > kMaxK) return fail(MF_ERR_K, "k=%d must be odd in [1, %d]", k, kMaxK);
    if (border != MF_BORDER_REPLICATE) return fail(MF_ERR_BORDER, "unknown border mode %d", border);
    return MF_OK;
}

int32_t median_filter_fwd_argmedian(const float* src, float* dst, int32_t* idx, int64_t planes, int64_t H,
                                    int64_t W, int32_t k, int32_t border, void* stream)
{
    g_last_error.clear();
    if (!src || !dst || !idx) return fail(MF_ERR_NULL, "src, dst or idx is NULL");
    int32_t rc = validate_planes(planes, H, W, k, border);
    if (rc) return rc;
    const size_t bytes = (size_t)(planes * H * W) * 4;
    if (overlap(src, bytes, dst, bytes) || overlap(src, bytes, idx, bytes) || overlap(dst, bytes, idx, bytes))
        return fail(MF_ERR_ALIAS, "src, dst and idx must not overlap");
    rc = median_filter_planes(src, dst, planes, H * W * 4, H, W, W * 4, MF_F32, k, border, nullptr, stream);
    if (rc) return rc;
    g_last_error.clear();
    return hip_status(mf_ag_argmedian_launch(src, dst, idx, planes, (int)H, (int)W, k, (hipStream_t)stream),
                      "argmedian kernel launch");
}

int32_t median_filter_bwd_gather(const float* grad_out, const int32_t* idx, float* grad_in, int64_t planes,
                                 int64_t H, int64_t W, int32_t k, int32_t border, void* stream)
{
    g_last_error.clear();
    if (!grad_out || !idx || !grad_in) return fail(MF_ERR_NULL, "grad_out, idx or grad_in is NULL");
    int32_t rc = validate_planes(planes, H, W, k, border);
    if (rc) return rc;
    const size_t bytes = (size_t)(planes * H * W) * 4;
    if (overlap(grad_in, bytes, grad_out, bytes) || overlap(grad_in, bytes, idx, bytes))
        return fail(MF_ERR_ALIAS, "grad_in overlaps an input");
    return hip_status(mf_ag_grad_launch(grad_out, idx, grad_in, planes, (int)H, (int)W, k, (hipStream_t)stream),
                      "gradient gather kernel launch");
}

int32_t mf_list_configs(int32_t dtype, int32_t k, mf_options* out, int32_t cap)
{
    g_last_error.clear();
    if (!elem_size(dtype)) return fail(MF_ERR_DTYPE, "unknown dtype %d", dtype);
    if (k < 1 || k % 2 == 0 || k > kMaxK) return fail(MF_ERR_K, "k=%d must be odd in [1, %d]", k, kMaxK);
    if (cap > 0 && !out) return fail(MF_ERR_NULL, "output array is NULL");
    int n = 0;
    if (k > 1) {
        for (int i = 0; i < kOblCount; ++i) {
            if (kOblTable[i].k != k) continue;
            if (n < cap) {
                out[n].variant = MF_VARIANT_OBLIVIOUS;
                out[n].tile_w = kOblTable[i].tw;
                out[n].tile_h = kOblTable[i].th;
                out[n].group = kOblTable[i].nw;
                out[n].form = kOblTable[i].form;
                out[n].rows = kOblTable[i].ry;
            }
            ++n;
        }
        int tw[32], th[32], gr[32], fm[32];
        const int m = mf_da_list(dtype, k, tw, th, gr, 32, fm);
        for (int i = 0; i < m && i < 32; ++i) {
            if (n < cap) {
                out[n].variant = MF_VARIANT_DATA_AWARE;
                out[n].tile_w = tw[i];
                out[n].tile_h = th[i];
                out[n].group = gr[i];
                out[n].form = fm[i];
                out[n].rows = 0;
            }
            ++n;
        }
    }
    return n;
}

int32_t mf_global_workspace(int32_t dtype, int32_t k, int32_t tile_w, int32_t tile_h, int64_t planes, int64_t H,
                            int64_t W, int64_t* slot_bytes, int64_t* all_bytes, mf_options* resolved)
{
    g_last_error.clear();
    if (!slot_bytes || !all_bytes) return fail(MF_ERR_NULL, "output pointer is NULL");
    if (!elem_size(dtype)) return fail(MF_ERR_DTYPE, "unknown dtype %d", dtype);
    if (k < 3 || k % 2 == 0 || k > kMaxK) return fail(MF_ERR_K, "k=%d must be odd in [3, %d]", k, kMaxK);
    if (planes < 1 || H < 1 || W < 1 || H > (1 << 30) || W > (1 << 30) || planes > ((int64_t)1 << 30))
        return fail(MF_ERR_DIMS, "planes=%lld H=%lld W=%lld outside [1, 2^30]", (long long)planes, (long long)H,
                    (long long)W);
    mf_options o = {};
    o.tile_w = tile_w;
    o.tile_h = tile_h;
    int32_t tw = 0, th = 0;
    int32_t rc = global_tile_option(k, &o, &tw, &th);
    if (rc) return rc;
    long long slot = 0, all = 0;
    int utw = 0, uth = 0;
    if (!mf_dag_workspace(dtype, k, tw, th, planes, (int)H, (int)W, &slot, &all, &utw, &uth))
        return fail(MF_ERR_CONFIG, "no global-memory schedule for k=%d tile %dx%d", k, tw, th);
    *slot_bytes = slot;
    *all_bytes = all;
    if (resolved) {
        mf_options r = {};
        r.variant = MF_VARIANT_GLOBAL;
        r.tile_w = utw;
        r.tile_h = uth;
        r.rows = mf_dag_passes(dtype, k, utw, uth);
        *resolved = r;
    }
    return MF_OK;
}

int32_t median_filter_global(const void* src, void* dst, int64_t planes, int64_t plane_stride_bytes, int64_t H,
                             int64_t W, int64_t pitch_bytes, int32_t dtype, int32_t k, int32_t border,
                             int32_t tile_w, int32_t tile_h, void* workspace, int64_t workspace_bytes, void* stream)
{
    g_last_error.clear();
    int32_t rc = validate(src, dst, H, W, pitch_bytes, dtype, k, border);
    if (rc) return rc;
    if (k < 3) return fail(MF_ERR_K, "the global-memory form needs k >= 3");
    rc = check_planes(src, dst, planes, &plane_stride_bytes, H, W, pitch_bytes, dtype);
    if (rc) return rc;
    mf_options o = {};
    o.tile_w = tile_w;
    o.tile_h = tile_h;
    int32_t tw = 0, th = 0;
    rc = global_tile_option(k, &o, &tw, &th);
    if (rc) return rc;
    long long slot = 0, all = 0;
    int utw = 0, uth = 0;
    if (!mf_dag_workspace(dtype, k, tw, th, planes, (int)H, (int)W, &slot, &all, &utw, &uth))
        return fail(MF_ERR_CONFIG, "no global-memory schedule for k=%d tile %dx%d", k, tw, th);
    if (!workspace) return fail(MF_ERR_NULL, "workspace is NULL");
    if ((uintptr_t)workspace % 256)
        return fail(MF_ERR_WORKSPACE, "workspace not aligned to 256 bytes");
    if (workspace_bytes < slot)
        return fail(MF_ERR_WORKSPACE, "workspace of %lld bytes is below one tile's %lld bytes",
                    (long long)workspace_bytes, slot);
    const int s = elem_size(dtype);
    const uintptr_t img = (uintptr_t)((planes - 1) * plane_stride_bytes + (H - 1) * pitch_bytes + W * s);
    const uintptr_t a0 = (uintptr_t)workspace, sa = (uintptr_t)src, da = (uintptr_t)dst;
    const uintptr_t wl = (uintptr_t)workspace_bytes;
    if ((a0 < sa + img && sa < a0 + wl) || (a0 < da + img && da < a0 + wl))
        return fail(MF_ERR_ALIAS, "workspace overlaps src or dst");
    return hip_status(mf_dag_launch(src, dst, (int)planes, plane_stride_bytes, (int)H, (int)W, pitch_bytes, dtype,
                                    k, tw, th, workspace, workspace_bytes, (hipStream_t)stream),
                      "global-memory kernel launch");
}

int32_t mf_max_k_3d(void) { return mf_da3_max_k(); }

int32_t median_filter_3d(const void* src, void* dst, int64_t D, int64_t H, int64_t W, int64_t pitch_bytes,
                         int64_t slice_bytes, int32_t dtype, int32_t k, int32_t border, void* stream)
{
    g_last_error.clear();
    // the single-plane checks (k = 1 stands in for the box in the k test)
    int32_t rc = validate(src, dst, H, W, pitch_bytes, dtype, 1, border);
    if (rc) return rc;
    const int s = elem_size(dtype);
    if (D < 1 || D > (1 << 30)) return fail(MF_ERR_DIMS, "D=%lld outside [1, 2^30]", (long long)D);
    if (k < 1 || k % 2 == 0 || k > mf_da3_max_k())
        return fail(MF_ERR_K, "k=%d must be odd in [1, %d] for a 3-D box", k, mf_da3_max_k());
    const int64_t plane = (H - 1) * pitch_bytes + W * s;
    if (D > 1 && (slice_bytes < plane || slice_bytes % s || slice_bytes > ((int64_t)1 << 46)))
        return fail(MF_ERR_PITCH, "slice stride %lld: slices of %lld bytes would overlap or misalign",
                    (long long)slice_bytes, (long long)plane);
    if (D == 1) slice_bytes = plane;
    const uintptr_t a0 = (uintptr_t)src, b0 = (uintptr_t)dst;
    const uintptr_t len = (uintptr_t)((D - 1) * slice_bytes + plane);
    if (a0 < b0 + len && b0 < a0 + len) return fail(MF_ERR_ALIAS, "src and dst volumes overlap");
    if (!mf_da3_supports(dtype, k) && k != 1)
        return fail(MF_ERR_CONFIG, "no 3-D schedule for k=%d", k);
    hipStream_t st = (hipStream_t)stream;
    if (k == 1) {
        for (int64_t z = 0; z < D; ++z) {
            rc = hip_status(hipMemcpy2DAsync((char*)dst + z * slice_bytes, pitch_bytes,
                                             (const char*)src + z * slice_bytes, pitch_bytes, W * s, H,
                                             hipMemcpyDeviceToDevice, st),
                            "hipMemcpy2DAsync");
            if (rc) return rc;
        }
        return MF_OK;
    }
    return hip_status(mf_da3_launch(src, dst, (int)D, (int)H, (int)W, pitch_bytes, slice_bytes, dtype, k, st),
                      "3-D kernel launch");
}

int32_t mf_max_k(void) { return kMaxK; }

const char* mf_status_string(int32_t status)
{
    switch (status) {
    case MF_OK: return "ok";
    case MF_ERR_NULL: return "null pointer";
    case MF_ERR_DIMS: return "bad image dimensions";
    case MF_ERR_PITCH: return "bad pitch";
    case MF_ERR_DTYPE: return "bad dtype";
    case MF_ERR_K: return "bad kernel diameter";
    case MF_ERR_BORDER: return "bad border mode";
    case MF_ERR_ALIAS: return "source and destination overlap";
    case MF_ERR_NOMEM: return "out of device memory";
    case MF_ERR_PLAN: return "bad plan";
    case MF_ERR_CONFIG: return "configuration not available";
    case MF_ERR_WORKSPACE: return "workspace too small or misaligned";
    case MF_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char* mf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
