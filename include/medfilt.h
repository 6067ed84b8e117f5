/*
 * medfilt.h -- C ABI of the MI355X (gfx950) hierarchical-tiling median filter.
 *
 * The operation (Sugy, "A Fast Parallel Median Filtering Algorithm Using
 * Hierarchical Tiling", SIGGRAPH 2025, Section 1): every output pixel is the
 * median of the k x k window centred on it. The library computes it exactly,
 * by hierarchical tiling (Section 3) in one of two GPU realisations: a
 * data-oblivious selection network held in registers (Section 4) and a
 * data-aware merge held in LDS (Section 5).
 *
 * Conventions shared by every entry point:
 *   - Images are single planes, row-major, H rows of W elements, consecutive
 *     rows pitch_bytes apart. src and dst are DEVICE pointers owned by the
 *     caller, share the pitch and must not overlap (MF_ERR_ALIAS).
 *   - pitch_bytes >= W * sizeof(element) and a multiple of sizeof(element);
 *     src and dst are aligned to sizeof(element) (MF_ERR_PITCH otherwise).
 *   - k is odd, 1 <= k <= mf_max_k(); k = 1 copies the image. k may exceed H
 *     or W. Border: replicate (coordinates are clamped into the image); the
 *     paper states no border rule, this is the reading the library takes.
 *   - dtype: MF_U8, MF_U16, MF_U32 compare as unsigned integers; MF_F32
 *     compares under IEEE 754 totalOrder on the bit pattern (-NaN < -inf <
 *     ... < -0 < +0 < ... < +inf < +NaN), so the output is bit-exact and
 *     defined for every input, NaNs and signed zeros included.
 *   - Every argument is validated on the host before any GPU work; a bad
 *     argument returns a negative mf_status and launches nothing.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     null stream). Launch failures return MF_ERR_HIP with a message in
 *     mf_last_error(). No call allocates device memory on the plain path.
 *   - No C++ exception or abort crosses this interface.
 */
#ifndef MEDFILT_H
#define MEDFILT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mf_dtype { MF_U8 = 0, MF_U16 = 1, MF_U32 = 2, MF_F32 = 3 };

enum mf_border { MF_BORDER_REPLICATE = 0 };

enum mf_variant {
    MF_VARIANT_AUTO = 0,       /* the library's per-(k, dtype) choice          */
    MF_VARIANT_OBLIVIOUS = 1,  /* register-resident selection network, Sec. 4 */
    MF_VARIANT_DATA_AWARE = 2, /* LDS-resident merges, Sec. 5                   */
    MF_VARIANT_GLOBAL = 3      /* data-aware, lists in device memory, run in
                                  passes of two recursion levels over slices of
                                  tiles (the multi-pass form of Sec. 5.3)       */
};

enum mf_status {
    MF_OK = 0,
    MF_ERR_NULL = -1,     /* a required pointer is NULL                       */
    MF_ERR_DIMS = -2,     /* H < 1, W < 1, or a size that overflows int32 math */
    MF_ERR_PITCH = -3,    /* pitch_bytes < W*size, not a multiple of size, or
                             a pointer not aligned to the element size       */
    MF_ERR_DTYPE = -4,    /* unknown dtype, or one the entry point refuses   */
    MF_ERR_K = -5,        /* k even, < 1 or > mf_max_k()                      */
    MF_ERR_BORDER = -6,   /* unknown border mode                              */
    MF_ERR_ALIAS = -7,    /* src and dst byte ranges overlap                  */
    MF_ERR_NOMEM = -8,    /* a plan could not allocate its device tables     */
    MF_ERR_PLAN = -9,     /* plan misuse (NULL plan, shape mismatch)          */
    MF_ERR_CONFIG = -10,  /* the requested variant or tile is not available  */
    MF_ERR_WORKSPACE = -11, /* a caller workspace below one tile's size, or
                               not 256-byte aligned                          */
    MF_ERR_HIP = -100     /* a HIP runtime call failed; see mf_last_error()  */
};

/* Options of median_filter_ex. Zero-initialise, then set what is needed. */
typedef struct mf_options {
    int32_t variant;  /* enum mf_variant                                     */
    int32_t tile_w;   /* root tile width, power of two <= k; 0 = library's   */
    int32_t tile_h;   /* root tile height, power of two <= k; 0 = library's  */
    int32_t group;    /* data-aware: root tiles per work-group (1, 2, 4);
                         oblivious: waves per work-group (1, 4);
                         0 = library's                                      */
    int32_t form;     /* oblivious: 1 = columns sorted once per work-group and
                         shared by the tiles, 2 = each tile sorts its own
                         columns (small k), 3 = column-strip streaming form
                         (k = 3 only: root tile 1x1, each sorted column
                         shared by three windows, rows streamed through
                         registers); 0 = library's                          */
    int32_t rows;     /* oblivious: tile rows per wave; 0 = library's       */
} mf_options;

/* k x k median of one plane (Section 1 definition, Section 3 method).
 * src, dst: device pointers to H rows of W elements of `dtype`, pitch_bytes
 * apart. Returns MF_OK once the kernels are enqueued on `stream`. */
int32_t median_filter(const void* src, void* dst, int64_t H, int64_t W,
                      int64_t pitch_bytes, int32_t dtype, int32_t k,
                      int32_t border, void* stream);

/* As median_filter, with the variant and root tile chosen by the caller
 * (opt may be NULL = defaults). A variant or tile the library was not built
 * for returns MF_ERR_CONFIG. Results are identical for every valid choice. */
int32_t median_filter_ex(const void* src, void* dst, int64_t H, int64_t W,
                         int64_t pitch_bytes, int32_t dtype, int32_t k,
                         int32_t border, const mf_options* opt, void* stream);

/* As median_filter_ex, over `planes` planes of H x W in one launch (the
 * channels of an image, a batch of equal-size images): plane p starts at
 * src/dst + p * plane_stride_bytes. Every plane is filtered separately (no
 * window crosses planes; the border rule applies per plane). planes = 1
 * ignores plane_stride_bytes; otherwise it must be a multiple of the element
 * size and at least (H-1)*pitch_bytes + W*element size (planes do not
 * overlap), and the src and dst ranges of all planes must not overlap
 * (MF_ERR_PITCH, MF_ERR_ALIAS). Filtering planes in one launch lets the
 * persistent kernels balance blocks across planes. */
int32_t median_filter_planes(const void* src, void* dst, int64_t planes,
                             int64_t plane_stride_bytes, int64_t H, int64_t W,
                             int64_t pitch_bytes, int32_t dtype, int32_t k,
                             int32_t border, const mf_options* opt, void* stream);

/* Median of a rectangular window: every output pixel is the median of the
 * kw x kh window centred on it (kw columns, kh rows, both odd), the
 * rectangular neighbourhood of the Section 1 definition; the tile terminology
 * of Section 3.2 (footprint (kw+t_w-1) x (kh+t_h-1), core
 * (kw-t_w+1) x (kh-t_h+1)) and the recursion of Section 3 carry over with
 * separate horizontal and vertical radii. Arguments, planes and errors as in
 * median_filter_planes. kw == kh is the square filter (median_filter_planes
 * with opt's variant and default tiles, any k up to mf_max_k()). A
 * rectangular window runs an oblivious network (Section 4) where one is
 * compiled for (kw, kh) and the data-aware variant (Section 5, one generated
 * schedule per shape) otherwise; both sides must lie in
 * [1, mf_max_rect_side()] (MF_ERR_K otherwise). opt may be NULL; for a
 * rectangular window only opt->variant is honoured (MF_VARIANT_AUTO,
 * MF_VARIANT_OBLIVIOUS: MF_ERR_CONFIG when no network is compiled for the
 * shape, MF_VARIANT_DATA_AWARE); any non-zero tile, group, form or rows is
 * MF_ERR_CONFIG. Results are identical for every variant. */
int32_t median_filter_rect(const void* src, void* dst, int64_t planes,
                           int64_t plane_stride_bytes, int64_t H, int64_t W,
                           int64_t pitch_bytes, int32_t dtype, int32_t kw, int32_t kh,
                           int32_t border, const mf_options* opt, void* stream);

/* Largest side of a rectangular (kw != kh) window median_filter_rect
 * accepts. */
int32_t mf_max_rect_side(void);

/* The variant and root tile median_filter_rect runs for (dtype, kw, kh):
 * kw == kh answers as mf_query_config with default options; otherwise
 * MF_VARIANT_OBLIVIOUS and the network's root tile when one is compiled for
 * the shape, else MF_VARIANT_DATA_AWARE and the generated schedule's tile
 * (the MF_VARIANT_AUTO choice). Errors as
 * median_filter_rect's window and dtype checks (MF_ERR_NULL for a NULL
 * output pointer). */
int32_t mf_query_rect_config(int32_t dtype, int32_t kw, int32_t kh, int32_t* variant,
                             int32_t* tile_w, int32_t* tile_h);

/* Diagnostic (not part of the filter): enqueue `blocks` work-groups of 256
 * threads, each thread running `iters` iterations of 256 dependent packed
 * 16-bit min/max instructions in 8 independent chains (512 element-ops per
 * iteration), and write one word per thread to `out` (a device buffer of
 * blocks*256 uint32). Timing it gives the measured min/max rate that the
 * oblivious networks' roofline is compared against. MF_ERR_DIMS for a NULL
 * buffer or non-positive sizes. */
int32_t mf_peak_minmax(void* out, int32_t blocks, int32_t iters, void* stream);

/* The configuration median_filter_ex would run for (dtype, k, opt): the
 * variant and root tile actually used. Host-only; no GPU needed. */
int32_t mf_query_config(int32_t dtype, int32_t k, const mf_options* opt,
                        int32_t* variant, int32_t* tile_w, int32_t* tile_h);

/* As mf_query_config, with every field of the configuration that runs:
 * variant, root tile, group (oblivious: waves per work-group; data-aware:
 * root tiles per work-group), form (oblivious column-sort form, 3 = the
 * k = 3 column-strip form) and rows (oblivious tile rows per wave); fields
 * that do not apply are 0. k = 1 (a copy) gives variant 0 and a 1x1 tile.
 * Host only. MF_ERR_NULL for a NULL `resolved`, other errors as
 * mf_query_config. */
int32_t mf_query_options(int32_t dtype, int32_t k, const mf_options* opt, mf_options* resolved);

/* ---- Global-memory multi-pass form ------------------------------------
 * The data-aware variant with its sorted lists in device memory instead of
 * LDS (Section 5.3: the global-memory realisation runs the recursion in
 * passes of two levels; Section 7.1: its memory need grows with the number
 * of tiles in flight). Every root tile's lists take one workspace slot of
 * slot_bytes; tiles run in slices of workspace_bytes / slot_bytes tiles, and
 * each slice runs the passes as successive launches, the lists staying in
 * their slots in between. The root tile is not bounded by the LDS (larger
 * tiles share more work per pixel). Square windows, 3 <= k <= mf_max_k(),
 * all four dtypes, results identical to median_filter. Through
 * median_filter_ex / median_filter_planes (opt->variant = MF_VARIANT_GLOBAL,
 * optional tile_w / tile_h) the library allocates the workspace (all tiles
 * at once, capped at 256 MiB) and frees it in stream order; this is the one
 * plain-path option that allocates device memory. */

/* Workspace sizes for `planes` planes of H x W with root tile tile_w x
 * tile_h (0 x 0 = the library's): *slot_bytes per tile in flight (the
 * minimum workspace), *all_bytes for every tile at once (one slice). When
 * resolved is not NULL it receives the variant, the root tile and, in
 * `rows`, the number of passes. Host only. MF_ERR_K for k < 3 or even,
 * MF_ERR_CONFIG for a tile without a schedule. */
int32_t mf_global_workspace(int32_t dtype, int32_t k, int32_t tile_w, int32_t tile_h,
                            int64_t planes, int64_t H, int64_t W,
                            int64_t* slot_bytes, int64_t* all_bytes, mf_options* resolved);

/* The global-memory form over `planes` planes (arguments and errors as
 * median_filter_planes, k >= 3) with a caller workspace: a device pointer,
 * 256-byte aligned, of workspace_bytes >= *slot_bytes (MF_ERR_WORKSPACE
 * otherwise), not overlapping src or dst (MF_ERR_ALIAS). Allocates nothing;
 * the workspace is in use until the work enqueued on `stream` completes. */
int32_t median_filter_global(const void* src, void* dst, int64_t planes,
                             int64_t plane_stride_bytes, int64_t H, int64_t W,
                             int64_t pitch_bytes, int32_t dtype, int32_t k, int32_t border,
                             int32_t tile_w, int32_t tile_h, void* workspace,
                             int64_t workspace_bytes, void* stream);

/* ---- 3-D boxes -----------------------------------------------------------
 * Median of the k x k x k box around every voxel of a volume (the extension
 * of hierarchical tiling to a third axis that Section 7.2 proposes for
 * medical imaging): the data-aware recursion with tiles of t_w x t_h x t_z
 * voxels, whose lists are a sorted core, faces (one per outside coordinate
 * on an axis), edges (one per pair of outside coordinates) and raw corners.
 * Each axis is clamped (replicate border). The volume has D slices of H rows
 * of W elements; rows are pitch_bytes apart, slices slice_bytes apart
 * (>= (H-1)*pitch_bytes + W*size and a multiple of the element size unless
 * D = 1), shared by src and dst, which must not overlap. k odd in
 * [1, mf_max_k_3d()]; k = 1 copies. Errors as median_filter_planes. */
int32_t median_filter_3d(const void* src, void* dst, int64_t D, int64_t H, int64_t W,
                         int64_t pitch_bytes, int64_t slice_bytes, int32_t dtype, int32_t k,
                         int32_t border, void* stream);

/* Largest k of median_filter_3d. */
int32_t mf_max_k_3d(void);

/* ---- Batched form -------------------------------------------------------
 * Many images of uneven sizes, kernel diameters and dtypes filtered by ONE
 * hipGraph launch. A plan groups its images by kernel (variant, k, root tile,
 * value class) and gives each group one kernel node whose grid covers all of
 * the group's images; the nodes run as parallel graph branches. Each image
 * follows the conventions of median_filter (k >= 3 here); no destination may
 * overlap another image's source or destination. */
typedef struct mf_image {
    const void* src;       /* device pointer */
    void* dst;             /* device pointer */
    int64_t H, W, pitch_bytes;
    int32_t dtype, k, border;
} mf_image;

typedef struct mf_plan_s* mf_plan;

/* Build a plan for n images: device job tables (one hipMalloc, owned by the
 * plan) and an instantiated graph. *plan is NULL on failure. */
int32_t mf_plan_create(const mf_image* imgs, int32_t n, mf_plan* plan);

/* Same images (shapes, pitches, dtypes, k) with new pointers. Waits for the
 * plan's last launch to finish (an event recorded by mf_plan_launch; other
 * work on the device is not waited for), then rewrites the job tables; the
 * graph is reused. */
int32_t mf_plan_update(mf_plan plan, const mf_image* imgs, int32_t n);

/* One graph launch on `stream` filtering every image of the plan. */
int32_t mf_plan_launch(mf_plan plan, void* stream);

/* Number of kernel groups and total work-groups of a plan (host only). */
int32_t mf_plan_info(mf_plan plan, int32_t* buckets, int64_t* blocks);

/* Free a plan (waits for the plan's last launch to finish). NULL is ignored. */
void mf_plan_destroy(mf_plan plan);

/* Create a plan, launch it on `stream`, wait for it, destroy it. */
int32_t median_filter_batched(const mf_image* imgs, int32_t n, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the batched form
 * without a plan. Same images, conventions and results as
 * median_filter_batched, but nothing is allocated: the per-image job records
 * go to a static device array of the library (MF_NOALLOC_MAX_IMAGES records
 * of 48 bytes, 192 KiB, one per GPU, held until the process ends), and the
 * kernels (one per group of images sharing a kernel, plus one small launch
 * per 64 records that writes the records) are enqueued on `stream`; the call
 * returns without waiting. n must be in [1, MF_NOALLOC_MAX_IMAGES]
 * (MF_ERR_DIMS otherwise); argument errors as mf_plan_create, before any GPU
 * work. Every call on one GPU shares that GPU's array and overwrites it:
 * calls that overlap on one GPU (other streams or threads) race, so the
 * caller must order them (the same stream orders them). */
#define MF_NOALLOC_MAX_IMAGES 4096
int32_t median_filter_batched_noalloc(const mf_image* imgs, int32_t n, void* stream);

/* Differentiable form, forward: median (as median_filter) and argmedian of
 * `planes` contiguous float32 planes of H x W (NCHW-style, plane stride H*W).
 * idx[p] is the plane-local flat index y*W + x of the input pixel the median
 * of p was taken from: among the pixels of p's clamped window whose bits equal
 * the median, the lowest flat index. The paper has no gradient; this tie rule
 * is the library's. src, dst and idx are device pointers that must not
 * overlap; H*W must be < 2^31. */
int32_t median_filter_fwd_argmedian(const float* src, float* dst, int32_t* idx, int64_t planes,
                                    int64_t H, int64_t W, int32_t k, int32_t border, void* stream);

/* Differentiable form, backward: grad_in[q] = sum of grad_out[p] over the
 * pixels p of the same plane with idx[p] == q, added in binary32 from +0 in
 * ascending p (bit-reproducible, no atomics). idx must come from
 * median_filter_fwd_argmedian with the same k. Device pointers, contiguous
 * planes, grad_in must not overlap the inputs. */
int32_t median_filter_bwd_gather(const float* grad_out, const int32_t* idx, float* grad_in, int64_t planes,
                                 int64_t H, int64_t W, int32_t k, int32_t border, void* stream);

/* Every compiled configuration for (dtype, k): writes up to `cap` entries to
 * out (variant, tile_w, tile_h, group all set) and returns how many exist, or
 * a negative mf_status. The first entry is the library's default. Host only;
 * this is what an autotuner enumerates. */
int32_t mf_list_configs(int32_t dtype, int32_t k, mf_options* out, int32_t cap);

/* Largest supported kernel diameter. */
int32_t mf_max_k(void);

/* Static description of a status code. */
const char* mf_status_string(int32_t status);

/* Detail of the last error on the calling thread ("" if none). */
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MEDFILT_H */
