// Batched form that allocates nothing: the same kernels as a batched plan,
// launched directly on the caller's stream, with the job tables of one call
// in a library-owned static device array instead of a hipMalloc'd buffer.
//
// Host side: the images are validated and grouped by kernel exactly as a plan
// groups them (variant, k, root tile, value class); every bucket's jobs are
// laid out contiguously in the static array. The job records reach the device
// as kernel arguments of a small copy kernel (64 records per launch), so no
// host buffer has to outlive the call and no runtime copy is queued; then one
// kernel per bucket runs over the records of its images.
//
// The static array is one per GPU and shared by every call on that GPU: a call
// overwrites the previous call's records, so calls that overlap on one GPU
// (concurrent streams or threads) race and must be ordered by the caller.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <mutex>

#include "mf_internal.h"

int32_t mf_internal_fail(int32_t code, const char* msg);
int32_t mf_internal_resolve(int32_t dtype, int32_t k, int32_t* variant, int32_t* tw, int32_t* th,
                            int32_t* group, MfBatchedKernel* obl_p16, MfBatchedKernel* obl_u32, int32_t* da_form);
int32_t mf_internal_check_images(const mf_image* imgs, int32_t n);
void mf_internal_batched_grids(int n, const MfBatchedKernel* kern, const long long* blocks, const int* k,
                                unsigned* grid);

// The job records of the last call on this GPU (MF_NOALLOC_MAX_IMAGES x 48
// bytes). In host code the name is only a symbol handle; kernels get the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) MfJob scratch[MF_NOALLOC_MAX_IMAGES];

namespace {

constexpr int kPackJobs = 64;            // records per copy launch (3 KB of arguments)
constexpr int kMaxDevices = 64;
constexpr int kMaxBuckets = 512;         // (variant, k, tile, class) combinations of one call

struct JobPack {
    MfJob j[kPackJobs];
};

struct NaBucket {
    int variant, k, tw, th, group, packed;   // packed: the kernel class of the bucket
    MfBatchedKernel kern;
    MfDaArgs da;
    int first, count;        // records [first, first + count) of the static array
    long long blocks;
};

std::mutex g_mu;                         // host tables below; one call at a time
MfJob* g_ptr[kMaxDevices];               // device address of `scratch`, per device
NaBucket g_buckets[kMaxBuckets];
int g_bucket_of[MF_NOALLOC_MAX_IMAGES];
MfJob g_jobs[MF_NOALLOC_MAX_IMAGES];
MfBatchedKernel g_kern[kMaxBuckets];     // per-bucket launch shapes of the call
long long g_blocks[kMaxBuckets];
int g_k[kMaxBuckets];
unsigned g_grid[kMaxBuckets];

int32_t hip_fail(hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return mf_internal_fail(MF_ERR_HIP, buf);
}

}  // namespace

// Copies n <= kPackJobs records from the kernel arguments to dst.
__global__ void __launch_bounds__(kPackJobs) mf_noalloc_put_jobs(MfJob* __restrict__ dst, JobPack p, int n)
{
    const int i = threadIdx.x;
    if (i < n) dst[i] = p.j[i];
}

extern "C" int32_t median_filter_batched_noalloc(const mf_image* imgs, int32_t n, void* stream)
{
    if (imgs && n > MF_NOALLOC_MAX_IMAGES) {
        char buf[128];
        snprintf(buf, sizeof buf, "%d images exceed the static job table of %d", n, MF_NOALLOC_MAX_IMAGES);
        return mf_internal_fail(MF_ERR_DIMS, buf);
    }
    int32_t rc = mf_internal_check_images(imgs, n);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return mf_internal_fail(MF_ERR_HIP, "device ordinal out of range");
    if (!g_ptr[dev]) {
        // once per device, with that device current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = (MfJob*)p;
    }
    MfJob* const base = g_ptr[dev];
    // group the images by kernel, in first-appearance order
    int nb = 0;
    for (int i = 0; i < n; ++i) {
        const mf_image& m = imgs[i];
        int32_t variant = 0, tw = 0, th = 0, group = 0, da_form = 0;
        MfBatchedKernel kp16 = {}, ku32 = {};
        rc = mf_internal_resolve(m.dtype, m.k, &variant, &tw, &th, &group, &kp16, &ku32, &da_form);
        if (rc) return rc;
        // kernel class: the oblivious kernels serve 8- and 16-bit data alike;
        // the data-aware kernels differ for 8-bit data (byte elements),
        // 16-bit and 32-bit data
        const int packed = variant == MF_VARIANT_DATA_AWARE
                               ? 8 + (m.dtype == MF_U8 ? 0 : m.dtype == MF_U16 ? 1 : 2) * 4 + da_form
                               : (m.dtype == MF_U8 || m.dtype == MF_U16) ? 1 : 0;
        int b = 0;
        while (b < nb && !(g_buckets[b].variant == variant && g_buckets[b].k == m.k && g_buckets[b].tw == tw &&
                           g_buckets[b].th == th && g_buckets[b].group == group && g_buckets[b].packed == packed))
            ++b;
        if (b == nb) {
            if (nb == kMaxBuckets) return mf_internal_fail(MF_ERR_DIMS, "too many distinct kernels in one call");
            NaBucket& B = g_buckets[nb++];
            memset(&B, 0, sizeof B);
            B.variant = variant;
            B.k = m.k;
            B.tw = tw;
            B.th = th;
            B.group = group;
            B.packed = packed;
            if (variant == MF_VARIANT_OBLIVIOUS) {
                B.kern = packed ? kp16 : ku32;
            } else {
                e = mf_da_batched(m.dtype, m.k, tw, th, group, &B.kern, &B.da, da_form);
                if (e != hipSuccess) return hip_fail(e, "data-aware batched kernel");
            }
        }
        g_bucket_of[i] = b;
        ++g_buckets[b].count;
    }
    // records: bucket after bucket, images in call order within a bucket
    int first = 0;
    for (int b = 0; b < nb; ++b) {
        g_buckets[b].first = first;
        first += g_buckets[b].count;
        g_buckets[b].count = 0;
        g_buckets[b].blocks = 0;
    }
    for (int i = 0; i < n; ++i) {
        NaBucket& B = g_buckets[g_bucket_of[i]];
        const mf_image& m = imgs[i];
        MfJob& j = g_jobs[B.first + B.count++];
        j.src = (const unsigned char*)m.src;
        j.dst = (unsigned char*)m.dst;
        j.pitch = m.pitch_bytes;
        j.H = (int)m.H;
        j.W = (int)m.W;
        j.dtype = m.dtype;
        j.nbx = (int)((m.W + B.kern.bw - 1) / B.kern.bw);
        const long long nby = (m.H + B.kern.bh - 1) / B.kern.bh;
        if (B.blocks > 0x7fffffffLL) return mf_internal_fail(MF_ERR_DIMS, "a bucket needs more than 2^31-1 work-groups");
        j.block_begin = (int)B.blocks;
        j.pad = 0;
        B.blocks += (long long)j.nbx * nby;
    }
    for (int b = 0; b < nb; ++b)
        if (g_buckets[b].blocks > 0x7fffffffLL)
            return mf_internal_fail(MF_ERR_DIMS, "a bucket needs more than 2^31-1 work-groups");
    for (int b = 0; b < nb; ++b) {
        g_kern[b] = g_buckets[b].kern;
        g_blocks[b] = g_buckets[b].blocks;
        g_k[b] = g_buckets[b].k;
    }
    mf_internal_batched_grids(nb, g_kern, g_blocks, g_k, g_grid);
    hipStream_t s = (hipStream_t)stream;
    for (int i0 = 0; i0 < n; i0 += kPackJobs) {
        const int cnt = n - i0 < kPackJobs ? n - i0 : kPackJobs;
        JobPack pack;
        memset(&pack, 0, sizeof pack);
        memcpy(pack.j, g_jobs + i0, sizeof(MfJob) * cnt);
        MfJob* dst = base + i0;
        void* args[] = {&dst, &pack, (void*)&cnt};
        e = hipLaunchKernel((const void*)mf_noalloc_put_jobs, dim3(1), dim3(kPackJobs), args, 0, s);
        if (e != hipSuccess) return hip_fail(e, "launch of the job-record copy");
    }
    for (int b = 0; b < nb; ++b) {
        NaBucket& B = g_buckets[b];
        MfJob* jobs = base + B.first;
        int njobs = B.count;
        int nblocks = (int)B.blocks;
        void* args_obl[] = {&jobs, &njobs, &nblocks};
        void* args_da[] = {&jobs, &njobs, &nblocks, &B.da};
        e = hipLaunchKernel(B.kern.fn, dim3(g_grid[b]), dim3(B.kern.threads),
                            B.variant == MF_VARIANT_OBLIVIOUS ? args_obl : args_da, B.kern.lds, s);
        if (e != hipSuccess) return hip_fail(e, "batched kernel launch");
    }
    return MF_OK;
}
