// Batched form: many images of uneven sizes, kernel diameters and dtypes
// filtered by one hipGraph launch.
//
// A plan groups its images into buckets that share a kernel (variant, k, root
// tile, value class). Each bucket gets a job table in device memory (one MfJob
// per image, with the index of its first block) and one kernel node over
// every block of every image of the bucket (one work-group per block; the
// kernel's grid-stride loop also runs smaller grids). The nodes have no dependencies, so the graph
// runs the buckets as parallel branches. Updating a plan with new pointers
// rewrites the job tables only; the graph is unchanged.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "mf_internal.h"

// Shared with mf_api.cpp.
int32_t mf_internal_validate(const void* src, const void* dst, int64_t H, int64_t W, int64_t pitch,
                             int32_t dtype, int32_t k, int32_t border);
int32_t mf_internal_fail(int32_t code, const char* msg);
int32_t mf_internal_resolve(int32_t dtype, int32_t k, int32_t* variant, int32_t* tw, int32_t* th,
                            int32_t* group, MfBatchedKernel* obl_p16, MfBatchedKernel* obl_u32, int32_t* da_form);

namespace {

struct Bucket {
    int variant, k, tw, th, group, packed;
    MfBatchedKernel kern;
    MfDaArgs da;
    std::vector<int> images;
    std::vector<MfJob> jobs;
    long long blocks = 0;
    MfJob* d_jobs = nullptr;
    int njobs = 0;
    int nblocks = 0;
};

int elem_size(int dtype) { return dtype == MF_U8 ? 1 : dtype == MF_U16 ? 2 : 4; }

int32_t hip_fail(hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return mf_internal_fail(MF_ERR_HIP, buf);
}

}  // namespace

struct mf_plan_s {
    std::vector<mf_image> imgs;
    std::vector<Bucket> buckets;
    void* d_buf = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;      // recorded after every launch of the plan
    bool launched = false;
    int device = 0;
};

static void plan_free(mf_plan_s* p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_buf) (void)hipFree(p->d_buf);
    if (p->done) (void)hipEventDestroy(p->done);
    delete p;
}

// Work-groups of the batched launches of one call: one per block. The
// kernels walk their blocks with a grid-stride loop and run with any smaller
// grid, but resident-sized grids were measured slower on a mixed batch (256
// images, 12 buckets: 4.98 ms with a full resident grid per bucket, 8.3 ms
// with the resident work-groups split between the buckets by estimated work,
// 3.9 ms with one work-group per block): the buckets run concurrently, and
// one work-group per block lets the hardware interleave all of them and
// balance blocks of unequal cost, while a persistent grid serialises or
// starves them.
void mf_internal_batched_grids(int n, const MfBatchedKernel* kern, const long long* blocks, const int* k,
                                unsigned* grid)
{
    (void)kern;
    (void)k;
    for (int b = 0; b < n; ++b) grid[b] = (unsigned)blocks[b];
}

int32_t mf_internal_check_images(const mf_image* imgs, int32_t n)
{
    if (!imgs) return mf_internal_fail(MF_ERR_NULL, "image list is NULL");
    if (n < 1) return mf_internal_fail(MF_ERR_DIMS, "a plan needs at least one image");
    for (int i = 0; i < n; ++i) {
        const mf_image& m = imgs[i];
        int32_t rc = mf_internal_validate(m.src, m.dst, m.H, m.W, m.pitch_bytes, m.dtype, m.k, m.border);
        if (rc) return rc;
        if (m.k == 1) return mf_internal_fail(MF_ERR_K, "k=1 (a copy) is not supported in a batched plan");
    }
    // every destination must be disjoint from every other image's buffers:
    // the buckets of one launch run concurrently
    for (int i = 0; i < n; ++i) {
        const uintptr_t d0 = (uintptr_t)imgs[i].dst;
        const uintptr_t dl = (uintptr_t)((imgs[i].H - 1) * imgs[i].pitch_bytes + imgs[i].W * elem_size(imgs[i].dtype));
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            const uintptr_t len = (uintptr_t)((imgs[j].H - 1) * imgs[j].pitch_bytes +
                                              imgs[j].W * elem_size(imgs[j].dtype));
            const uintptr_t s0 = (uintptr_t)imgs[j].src, e0 = (uintptr_t)imgs[j].dst;
            if ((d0 < s0 + len && s0 < d0 + dl) || (d0 < e0 + len && e0 < d0 + dl)) {
                char buf[128];
                snprintf(buf, sizeof buf, "destination of image %d overlaps image %d", i, j);
                return mf_internal_fail(MF_ERR_ALIAS, buf);
            }
        }
    }
    return MF_OK;
}

static void fill_jobs(mf_plan_s* p)
{
    for (Bucket& b : p->buckets) {
        b.jobs.clear();
        long long next = 0;
        for (int i : b.images) {
            const mf_image& m = p->imgs[i];
            MfJob j;
            j.src = (const unsigned char*)m.src;
            j.dst = (unsigned char*)m.dst;
            j.pitch = m.pitch_bytes;
            j.H = (int)m.H;
            j.W = (int)m.W;
            j.dtype = m.dtype;
            j.nbx = (int)((m.W + b.kern.bw - 1) / b.kern.bw);
            const int nby = (int)((m.H + b.kern.bh - 1) / b.kern.bh);
            j.block_begin = (int)next;
            j.pad = 0;
            next += (long long)j.nbx * nby;
            b.jobs.push_back(j);
        }
        b.blocks = next;
        b.njobs = (int)b.jobs.size();
    }
}

static int32_t upload_jobs(mf_plan_s* p)
{
    for (Bucket& b : p->buckets) {
        hipError_t e = hipMemcpy(b.d_jobs, b.jobs.data(), sizeof(MfJob) * b.jobs.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(job table)");
    }
    return MF_OK;
}

extern "C" {

int32_t mf_plan_create(const mf_image* imgs, int32_t n, mf_plan* out)
{
    if (!out) return mf_internal_fail(MF_ERR_NULL, "plan output pointer is NULL");
    *out = nullptr;
    int32_t rc = mf_internal_check_images(imgs, n);
    if (rc) return rc;
    mf_plan_s* p = new (std::nothrow) mf_plan_s;
    if (!p) return mf_internal_fail(MF_ERR_NOMEM, "host allocation failed");
    p->imgs.assign(imgs, imgs + n);
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipGetDevice");
    }
    // bucket by kernel
    std::map<std::tuple<int, int, int, int, int>, int> index;
    for (int i = 0; i < n; ++i) {
        const mf_image& m = imgs[i];
        int32_t variant = 0, tw = 0, th = 0, group = 0, da_form = 0;
        MfBatchedKernel kp16 = {}, ku32 = {};
        rc = mf_internal_resolve(m.dtype, m.k, &variant, &tw, &th, &group, &kp16, &ku32, &da_form);
        if (rc) {
            plan_free(p);
            return rc;
        }
        const int packed = (m.dtype == MF_U8 || m.dtype == MF_U16) ? 1 : 0;
        // kernel class: the oblivious kernels serve 8- and 16-bit data alike;
        // the data-aware kernels differ for 8-bit data (byte elements),
        // 16-bit and 32-bit data
        const int cls = variant == MF_VARIANT_DATA_AWARE ? (m.dtype == MF_U8 ? 0 : m.dtype == MF_U16 ? 1 : 2) * 4 + da_form
                                                         : packed;
        auto key = std::make_tuple(variant, m.k, tw * 8 + group, th, cls);
        auto it = index.find(key);
        if (it == index.end()) {
            Bucket b;
            b.variant = variant;
            b.k = m.k;
            b.tw = tw;
            b.th = th;
            b.group = group;
            b.packed = packed;
            memset(&b.da, 0, sizeof b.da);
            if (variant == MF_VARIANT_OBLIVIOUS) {
                b.kern = packed ? kp16 : ku32;
            } else {
                e = mf_da_batched(m.dtype, m.k, tw, th, group, &b.kern, &b.da, da_form);
                if (e != hipSuccess) {
                    plan_free(p);
                    return hip_fail(e, "data-aware batched kernel");
                }
            }
            it = index.emplace(key, (int)p->buckets.size()).first;
            p->buckets.push_back(b);
        }
        p->buckets[it->second].images.push_back(i);
    }
    fill_jobs(p);
    size_t bytes = 0;
    for (Bucket& b : p->buckets) {
        if (b.blocks > 0x7fffffffLL) {
            plan_free(p);
            return mf_internal_fail(MF_ERR_DIMS, "a bucket needs more than 2^31-1 work-groups");
        }
        bytes += sizeof(MfJob) * b.jobs.size();
    }
    e = hipMalloc(&p->d_buf, bytes);
    if (e != hipSuccess) {
        plan_free(p);
        return mf_internal_fail(MF_ERR_NOMEM, "hipMalloc of the job tables failed");
    }
    size_t off = 0;
    for (Bucket& b : p->buckets) {
        b.d_jobs = (MfJob*)((char*)p->d_buf + off);
        off += sizeof(MfJob) * b.jobs.size();
    }
    rc = upload_jobs(p);
    if (rc) {
        plan_free(p);
        return rc;
    }
    e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipEventCreateWithFlags");
    }
    e = hipGraphCreate(&p->graph, 0);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipGraphCreate");
    }
    std::vector<MfBatchedKernel> kerns;
    std::vector<long long> nblk;
    std::vector<int> kk;
    for (Bucket& b : p->buckets) {
        kerns.push_back(b.kern);
        nblk.push_back(b.blocks);
        kk.push_back(b.k);
    }
    std::vector<unsigned> grids(p->buckets.size());
    mf_internal_batched_grids((int)p->buckets.size(), kerns.data(), nblk.data(), kk.data(), grids.data());
    size_t bi = 0;
    for (Bucket& b : p->buckets) {
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof kp);
        kp.func = (void*)b.kern.fn;
        kp.gridDim = dim3(grids[bi++]);
        kp.blockDim = dim3(b.kern.threads);
        kp.sharedMemBytes = (unsigned)b.kern.lds;
        b.nblocks = (int)b.blocks;
        void* args_obl[] = {&b.d_jobs, &b.njobs, &b.nblocks};
        void* args_da[] = {&b.d_jobs, &b.njobs, &b.nblocks, &b.da};
        kp.kernelParams = b.variant == MF_VARIANT_OBLIVIOUS ? args_obl : args_da;
        kp.extra = nullptr;
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, p->graph, nullptr, 0, &kp);
        if (e != hipSuccess) {
            plan_free(p);
            return hip_fail(e, "hipGraphAddKernelNode");
        }
    }
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = p;
    return MF_OK;
}

int32_t mf_plan_update(mf_plan p, const mf_image* imgs, int32_t n)
{
    if (!p) return mf_internal_fail(MF_ERR_PLAN, "plan is NULL");
    int32_t rc = mf_internal_check_images(imgs, n);
    if (rc) return rc;
    if (n != (int32_t)p->imgs.size()) return mf_internal_fail(MF_ERR_PLAN, "image count differs from the plan");
    for (int i = 0; i < n; ++i) {
        const mf_image &a = imgs[i], &b = p->imgs[i];
        if (a.H != b.H || a.W != b.W || a.pitch_bytes != b.pitch_bytes || a.dtype != b.dtype || a.k != b.k ||
            a.border != b.border)
            return mf_internal_fail(MF_ERR_PLAN, "image shape, pitch, dtype or k differs from the plan");
    }
    // the job tables may be in use by a launch still running: wait for the
    // plan's last launch only (other work on the device goes on)
    if (p->launched) {
        hipError_t e = hipEventSynchronize(p->done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    p->imgs.assign(imgs, imgs + n);
    fill_jobs(p);
    return upload_jobs(p);
}

int32_t mf_plan_launch(mf_plan p, void* stream)
{
    if (!p) return mf_internal_fail(MF_ERR_PLAN, "plan is NULL");
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    e = hipEventRecord(p->done, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->launched = true;
    return MF_OK;
}

void mf_plan_destroy(mf_plan p)
{
    if (!p) return;
    if (p->launched) (void)hipEventSynchronize(p->done);   // the plan's last launch, nothing else
    plan_free(p);
}

int32_t mf_plan_info(mf_plan p, int32_t* buckets, int64_t* blocks)
{
    if (!p || !buckets || !blocks) return mf_internal_fail(MF_ERR_NULL, "NULL argument");
    *buckets = (int32_t)p->buckets.size();
    long long t = 0;
    for (const Bucket& b : p->buckets) t += b.blocks;
    *blocks = t;
    return MF_OK;
}

int32_t median_filter_batched(const mf_image* imgs, int32_t n, void* stream)
{
    mf_plan p = nullptr;
    int32_t rc = mf_plan_create(imgs, n, &p);
    if (rc) return rc;
    rc = mf_plan_launch(p, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    mf_plan_destroy(p);
    if (rc) return rc;
    return e == hipSuccess ? MF_OK : hip_fail(e, "hipStreamSynchronize");
}

}  // extern "C"
