// Internal declarations shared by the dispatcher and the kernel translation
// units. Not part of the public ABI (include/medfilt.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "medfilt.h"

// Launcher of one compiled kernel configuration: `planes` planes of H x W,
// plane p at src/dst + p * plane_stride bytes. src/dst are device pointers,
// pitch in bytes, dtype an mf_dtype the kernel's value class accepts (u8/u16
// for the packed 16-bit class, u32/f32 for the 32-bit one).
typedef hipError_t (*mf_launch_fn)(const void* src, void* dst, int planes, long long plane_stride, int H,
                                   int W, long long pitch, int dtype, hipStream_t stream);

// One image of a batched launch. Images of one job table share the kernel
// (k, root tile, value class); block_begin is the first grid block of the
// image, ascending over the table.
struct MfJob {
    const unsigned char* src;
    unsigned char* dst;
    long long pitch;
    int H, W, dtype, nbx, block_begin, pad;
};

// A batched kernel: function, launch shape, and the output block of one
// work-group (bw x bh pixels; an image needs ceil(W/bw) x ceil(H/bh) blocks).
struct MfBatchedKernel {
    const void* fn;
    int threads;
    size_t lds;
    int bw, bh;
};

#define MF_OBL_NAME(NET, RY, NW, VC) mf_obl_launch_##NET##_r##RY##w##NW##_##VC
#define MF_OBL_BATCHED_NAME(NET, RY, NW, VC) mf_obl_batched_##NET##_r##RY##w##NW##_##VC

#define MF_OBL_DECLARE(NET, RY, NW)                                                \
    hipError_t MF_OBL_NAME(NET, RY, NW, p16)(const void*, void*, int, long long, int, int, \
                                             long long, int, hipStream_t);        \
    hipError_t MF_OBL_NAME(NET, RY, NW, u32)(const void*, void*, int, long long, int, int, \
                                             long long, int, hipStream_t);        \
    void MF_OBL_BATCHED_NAME(NET, RY, NW, p16)(MfBatchedKernel*);                 \
    void MF_OBL_BATCHED_NAME(NET, RY, NW, u32)(MfBatchedKernel*);

// Column-strip form for k = 3 (mf_strip.hip), per value class.
hipError_t mf_strip3_launch_p16(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                                long long pitch, int dtype, hipStream_t stream);
hipError_t mf_strip3_launch_u32(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                                long long pitch, int dtype, hipStream_t stream);

// Data-aware launcher: one per value class, any k up to mf_max_k(). kh = 0 is
// the square k x k window; otherwise the window is k columns by kh rows (a
// generated rectangular shape, both sides odd and at most
// mf_da_rect_max_side()).
// form: 0 = the default round mode of the entry found, 1 = rounds per
// recursion level, 2 = rounds over the whole schedule.
hipError_t mf_da_launch(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                        long long pitch, int dtype, int k, int tw, int th, int group, hipStream_t stream,
                        int kh = 0, int form = 0);
bool mf_da_supports(int dtype, int k, int tw, int th, int group, int kh = 0, int form = 0);
int mf_da_rect_max_side();
void mf_da_default_tile(int dtype, int k, int* tw, int* th, int* group, int kh = 0, int* form = nullptr);
// Data-aware entries for (dtype, k): fills up to cap (tw, th, group[, form])
// tuples, returns the count.
int mf_da_list(int dtype, int k, int* tw, int* th, int* group, int cap, int* form = nullptr);
// Batched data-aware kernel for (dtype class, k, tile); the blob pointer and
// schedule offsets are filled into *args (see mf_da_batched_args).
struct MfDaArgs {
    const uint32_t* blob;
    int k, kh, tw, th, c_off, r_off, nrounds, o_off, arena;   // window k columns x kh rows
    int groups;   // lane groups per work-group, each with its own root tiles
    int kz, tz;   // 3-D boxes: box depth and root tile depth (1 for planes)
};
hipError_t mf_da_batched(int dtype, int k, int tw, int th, int group, MfBatchedKernel* kern, MfDaArgs* args,
                         int form = 0);

// Global-memory multi-pass data-aware form: square k, root tile tw x th (0 =
// the library's), lists in a caller workspace of ws_bytes (device pointer,
// 256-byte aligned). Tiles run in slices of ws_bytes / slot_bytes, each
// slice in passes of two recursion levels (one launch per pass).
bool mf_dag_supports(int dtype, int k, int tw, int th);
bool mf_dag_workspace(int dtype, int k, int tw, int th, long long planes, int H, int W, long long* slot_bytes,
                      long long* all_bytes, int* used_tw, int* used_th);
int mf_dag_passes(int dtype, int k, int tw, int th);
hipError_t mf_dag_launch(const void* src, void* dst, int planes, long long plane_stride, int H, int W,
                         long long pitch, int dtype, int k, int tw, int th, void* ws, long long ws_bytes,
                         hipStream_t stream);

// 3-D box median, cubic k x k x k (mf_da3_supports): one kernel launch over
// a D x H x W volume, rows pitch bytes apart, slices slice bytes apart.
bool mf_da3_supports(int dtype, int k);
int mf_da3_max_k();
void mf_da3_tile(int dtype, int k, int* tw, int* th, int* tz);
hipError_t mf_da3_launch(const void* src, void* dst, int D, int H, int W, long long pitch, long long slice, int dtype,
                         int k, hipStream_t stream);

// Differentiable form (mf_autograd.hip).
hipError_t mf_ag_argmedian_launch(const float* src, const float* med, int32_t* idx, int64_t planes, int H,
                                  int W, int k, hipStream_t stream);
hipError_t mf_ag_grad_launch(const float* gout, const int32_t* idx, float* gin, int64_t planes, int H, int W,
                             int k, hipStream_t stream);
