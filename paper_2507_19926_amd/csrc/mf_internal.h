// Internal declarations shared by the dispatcher and the kernel translation
// units. Not part of the public ABI (include/medfilt.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "medfilt.h"

// Launcher of one compiled kernel configuration. src/dst are device
// pointers, pitch in bytes, dtype an mf_dtype the kernel's value class
// accepts (u8/u16 for the packed 16-bit class, u32/f32 for the 32-bit one).
typedef hipError_t (*mf_launch_fn)(const void* src, void* dst, int H, int W,
                                   long long pitch, int dtype, hipStream_t stream);

#define MF_OBL_NAME(K, TW, TH, VC) mf_obl_launch_MfNet_k##K##_##TW##x##TH##_##VC

#define MF_OBL_DECLARE(K, TW, TH, RY)                                          \
    hipError_t MF_OBL_NAME(K, TW, TH, p16)(const void*, void*, int, int,       \
                                           long long, int, hipStream_t);       \
    hipError_t MF_OBL_NAME(K, TW, TH, u32)(const void*, void*, int, int,       \
                                           long long, int, hipStream_t);

// Data-aware launcher: one per value class, any k up to mf_max_k().
hipError_t mf_da_launch(const void* src, void* dst, int H, int W, long long pitch,
                        int dtype, int k, int tw, int th, hipStream_t stream);
bool mf_da_supports(int dtype, int k, int tw, int th);
void mf_da_default_tile(int dtype, int k, int* tw, int* th);
