// Batched rendering of many requests over several resident trees in one
// persistent launch: every wave pulls 8x8 tiles from a shared counter until
// the launch's tile range is exhausted (every wave reaches that exit).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "dot_device.h"

namespace dot {

// Device record of one job: a contiguous range of one image's tiles.
struct JobDev {
    TreeView tv;
    const dot_camera* cam;
    float* rgb;
    int64_t tile_begin;     // first tile of the image rendered by this job
    int32_t width, height;
    int32_t storage, degree;
    float bg[3];
    float thr;
};

// Render one tile of one job (all lanes of the wave share the job).
template <int DT, int DEG>
__device__ __forceinline__ void tile_job(const JobDev& j, int64_t local_tile, int lane, int* stk) {
    const int tw = (j.width + 7) >> 3;
    const int64_t t = j.tile_begin + local_tile;
    const int ty = (int)(t / tw), tx = (int)(t - (int64_t)ty * tw);
    const int u = tx * 8 + (lane & 7), v = ty * 8 + (lane >> 3);
    if (u >= j.width || v >= j.height) return;
    Ray r = camera_ray(*j.cam, u, v);
    FwdArgs a{};
    a.thr = j.thr;
    FwdSeg<DT, DEG> seg(j.tv, a);
    sh_basis<DEG>((float)r.dx, (float)r.dy, (float)r.dz, seg.Y);
    int desc = 0;
    traverse(j.tv, r, stk, seg, desc);
    float* o = j.rgb + 3 * ((int64_t)v * j.width + u);
    o[0] = fmaf(seg.T, j.bg[0], seg.C[0]);
    o[1] = fmaf(seg.T, j.bg[1], seg.C[1]);
    o[2] = fmaf(seg.T, j.bg[2], seg.C[2]);
}

template <int DT>
__device__ __forceinline__ void tile_dt(const JobDev& j, int64_t lt, int lane, int* stk) {
    switch (j.degree) {
        case 0: tile_job<DT, 0>(j, lt, lane, stk); break;
        case 1: tile_job<DT, 1>(j, lt, lane, stk); break;
        case 2: tile_job<DT, 2>(j, lt, lane, stk); break;
        default: tile_job<DT, 3>(j, lt, lane, stk); break;
    }
}

// jobs[n_jobs], prefix[n_jobs + 1] (tile offsets of each job in this launch),
// counter: zero at launch.
__global__ __launch_bounds__(BLOCK) void render_jobs_kernel(const JobDev* __restrict__ jobs,
                                                            const int64_t* __restrict__ prefix, int n_jobs,
                                                            unsigned long long* __restrict__ counter) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t total = prefix[n_jobs];
    while (true) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(counter, 1ull);
        t = __shfl(t, 0, WAVE);
        if ((int64_t)t >= total) break;
        // job holding tile t: the last job whose prefix is <= t (wave-uniform search)
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= (int64_t)t) lo = mid;
            else hi = mid - 1;
        }
        const JobDev& j = jobs[lo];
        const int64_t lt = (int64_t)t - prefix[lo];
        switch (j.storage) {
            case DOT_F32: tile_dt<DOT_F32>(j, lt, lane, &stack_lds[tid]); break;
            case DOT_F16: tile_dt<DOT_F16>(j, lt, lane, &stack_lds[tid]); break;
            case DOT_PAL16: tile_dt<DOT_PAL16>(j, lt, lane, &stack_lds[tid]); break;
            default: tile_dt<DOT_BF16>(j, lt, lane, &stack_lds[tid]); break;
        }
    }
}

// Job tables reach the device through a ring of pinned host buffers, so the
// upload is asynchronous; a slot is reused only after its last copy finished.
namespace {
struct StageRing {
    static constexpr int N = 8;
    void* host[N] = {};
    size_t cap[N] = {};
    hipEvent_t ev[N] = {};
    bool used[N] = {};
    int next = 0;
    std::mutex m;
};
StageRing g_ring;
}  // namespace

static int stage_upload(const void* src, size_t bytes, void* dst, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_ring.m);
    int k = g_ring.next;
    g_ring.next = (k + 1) % StageRing::N;
    hipError_t e = hipSuccess;
    if (!g_ring.ev[k]) e = hipEventCreateWithFlags(&g_ring.ev[k], hipEventDisableTiming);
    if (e == hipSuccess && g_ring.used[k]) e = hipEventSynchronize(g_ring.ev[k]);
    if (e == hipSuccess && g_ring.cap[k] < bytes) {
        if (g_ring.host[k]) (void)hipHostFree(g_ring.host[k]);
        g_ring.host[k] = nullptr;
        g_ring.cap[k] = 0;
        size_t c = bytes < 4096 ? 4096 : bytes;
        e = hipHostMalloc(&g_ring.host[k], c, hipHostMallocDefault);
        if (e == hipSuccess) g_ring.cap[k] = c;
    }
    if (e == hipSuccess) {
        std::memcpy(g_ring.host[k], src, bytes);
        e = hipMemcpyAsync(dst, g_ring.host[k], bytes, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipEventRecord(g_ring.ev[k], s);
    if (e != hipSuccess) return hip_fail(e, "dot_render_jobs: job table upload");
    g_ring.used[k] = true;
    return DOT_OK;
}

size_t jobs_workspace_bytes(int n_jobs) {
    size_t b = sizeof(unsigned long long) * 2;                  // counter (+pad)
    b += sizeof(int64_t) * (size_t)(n_jobs + 1);                // prefix
    b = (b + 255) & ~(size_t)255;
    b += sizeof(JobDev) * (size_t)n_jobs;
    return b;
}

int launch_render_jobs(const dot_render_job* jobs, int n_jobs, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t need = jobs_workspace_bytes(n_jobs);
    if (ws_bytes < need) return fail(DOT_EINVAL, "dot_render_jobs: workspace too small");
    // host image of the workspace: counter | prefix | jobs
    std::vector<unsigned char> host(need, 0);
    int64_t* prefix = reinterpret_cast<int64_t*>(host.data() + sizeof(unsigned long long) * 2);
    size_t jobs_off = (sizeof(unsigned long long) * 2 + sizeof(int64_t) * (size_t)(n_jobs + 1) + 255) & ~(size_t)255;
    JobDev* jd = reinterpret_cast<JobDev*>(host.data() + jobs_off);
    int64_t acc = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const dot_render_job& q = jobs[i];
        if (!q.tree || !q.cam || !q.rgb_out) return fail(DOT_EINVAL, "dot_render_jobs: job with a NULL tree, camera or output");
        if (q.width <= 0 || q.height <= 0) return fail(DOT_EINVAL, "dot_render_jobs: job with a non-positive size");
        int64_t nt = (int64_t)((q.width + 7) / 8) * ((q.height + 7) / 8);
        if (q.tile_begin < 0 || q.tile_count < 0 || q.tile_begin + q.tile_count > nt)
            return fail(DOT_EINVAL, "dot_render_jobs: tile range outside the image");
        if (!(q.t_stop >= 0.f && q.t_stop < 1.f)) return fail(DOT_EINVAL, "dot_render_jobs: t_stop must be in [0, 1)");
        prefix[i] = acc;
        acc += q.tile_count;
        JobDev& d = jd[i];
        d.tv = q.tree->view();
        d.cam = q.cam;
        d.rgb = q.rgb_out;
        d.tile_begin = q.tile_begin;
        d.width = q.width;
        d.height = q.height;
        d.storage = q.tree->storage;
        d.degree = q.tree->degree;
        for (int a = 0; a < 3; ++a) d.bg[a] = q.bg[a];
        d.thr = q.t_stop > 0.f ? -std::log(q.t_stop) : __builtin_huge_valf();
    }
    prefix[n_jobs] = acc;
    if (acc == 0) return DOT_OK;
    int rc = stage_upload(host.data(), need, ws, s);
    if (rc) return rc;
    static int grid = 0;
    if (grid == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, render_jobs_kernel, BLOCK, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            per_cu = 2;
            cus = 256;
        }
        grid = (per_cu < 1 ? 1 : per_cu) * cus;
    }
    int64_t want = (acc + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    unsigned g = (unsigned)(want < grid ? want : grid);
    unsigned char* base = static_cast<unsigned char*>(ws);
    hipLaunchKernelGGL(render_jobs_kernel, dim3(g), dim3(BLOCK), 0, s,
                       reinterpret_cast<const JobDev*>(base + jobs_off),
                       reinterpret_cast<const int64_t*>(base + sizeof(unsigned long long) * 2), n_jobs,
                       reinterpret_cast<unsigned long long*>(base));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "dot_render_jobs: launch");
    return DOT_OK;
}

}  // namespace dot
