// Batched rendering of many requests over several resident trees in one
// persistent launch.  The launch's tiles are cut into 8 contiguous chunks, one
// per XCD; a wave pulls 8x8 tiles from its own XCD's chunk through that
// chunk's counter, so neighbouring tiles share that XCD's L2, and once the
// chunk is drained moves on to the next chunks in turn (work stealing).  A
// wave leaves after finding all 8 chunks drained, so every wave exits.
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
    // tile index within the image: below (width/8 + 1) * (height/8 + 1), so 32-bit
    const int t = (int)(j.tile_begin + local_tile);
    const int ty = t / tw, tx = t - ty * tw;
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

// One launch per storage type present in a batch, so each launch has the
// registers -- hence the occupancy -- of its own leaf type; the SH degree is
// taken from the job (wave-uniform).
// jobs[n_jobs], prefix[n_jobs + 1] (tile offsets of each job in this launch),
// counters[8 * CTR_STRIDE]: tiles taken so far from each chunk (zero at
// launch), one cache line apart so the XCDs' atomics do not queue on one line.
// Workgroups are dispatched round-robin over the 8 XCDs, so workgroup b runs
// on XCD b mod 8 and starts with that chunk.
constexpr int JOB_CHUNKS = 8;
constexpr int CTR_STRIDE = 16;   // 64-bit counters per 128-byte line
constexpr int JOB_KINDS = 4;     // storage types

template <int DT>
__global__ __launch_bounds__(BLOCK) void render_jobs_kernel(const JobDev* __restrict__ jobs,
                                                            const int64_t* __restrict__ prefix, int n_jobs,
                                                            unsigned long long* __restrict__ counters) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t total = prefix[n_jobs];
    const int64_t chunk = (total + JOB_CHUNKS - 1) / JOB_CHUNKS;
    const int x0 = (int)(blockIdx.x & (JOB_CHUNKS - 1));
    int tried = 0;
    while (tried < JOB_CHUNKS) {
        const int x = (x0 + tried) & (JOB_CHUNKS - 1);
        const int64_t begin = (int64_t)x * chunk;
        const int64_t end = begin + chunk < total ? begin + chunk : total;
        unsigned long long* ctr = counters + x * CTR_STRIDE;
        // a drained chunk is recognised by a plain read (counters only grow,
        // so a stale read can only lead to one more attempt)
        const unsigned long long seen = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t seen_lo = __builtin_amdgcn_readfirstlane((uint32_t)seen);
        const uint32_t seen_hi = __builtin_amdgcn_readfirstlane((uint32_t)(seen >> 32));
        if ((int64_t)(((uint64_t)seen_hi << 32) | seen_lo) >= end - begin) {
            ++tried;
            continue;
        }
        unsigned long long k = 0;
        if (lane == 0) k = atomicAdd(ctr, 1ull);
        // lane 0's value, read as a wave-uniform (scalar) value, so the job
        // lookup and the job record stay in scalar registers
        const uint32_t k_lo = __builtin_amdgcn_readfirstlane((uint32_t)k);
        const uint32_t k_hi = __builtin_amdgcn_readfirstlane((uint32_t)(k >> 32));
        const int64_t t = begin + (int64_t)(((uint64_t)k_hi << 32) | k_lo);
        if (t >= end) {
            ++tried;          // chunk drained: steal from the next one
            continue;
        }
        // job holding tile t: the last job whose prefix is <= t (wave-uniform search)
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const JobDev& j = jobs[lo];
        const int64_t lt = t - prefix[lo];
        switch (j.degree) {
            case 0: tile_job<DT, 0>(j, lt, lane, &stack_lds[tid]); break;
            case 1: tile_job<DT, 1>(j, lt, lane, &stack_lds[tid]); break;
            case 2: tile_job<DT, 2>(j, lt, lane, &stack_lds[tid]); break;
            default: tile_job<DT, 3>(j, lt, lane, &stack_lds[tid]); break;
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

// Workspace layout: counters [JOB_KINDS][8][CTR_STRIDE] | prefix (per storage type, n_k + 1
// entries each, types in order) | jobs sorted by storage type.
size_t jobs_workspace_bytes(int n_jobs) {
    size_t b = sizeof(unsigned long long) * JOB_KINDS * JOB_CHUNKS * CTR_STRIDE;
    b += sizeof(int64_t) * (size_t)(n_jobs + JOB_KINDS);
    b = (b + 255) & ~(size_t)255;
    b += sizeof(JobDev) * (size_t)n_jobs;
    return b;
}

namespace {

template <int DT>
hipError_t launch_kind(const JobDev* jobs, const int64_t* prefix, int n, int64_t tiles, unsigned long long* counters,
                       hipStream_t s) {
    // resident workgroups of this instantiation, found once
    static int grid = 0;
    if (grid == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, render_jobs_kernel<DT>, BLOCK, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            per_cu = 2;
            cus = 256;
        }
        grid = (per_cu < 1 ? 1 : per_cu) * cus;
    }
    const int64_t want = (tiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    const unsigned g = (unsigned)(want < grid ? want : grid);
    hipLaunchKernelGGL(render_jobs_kernel<DT>, dim3(g), dim3(BLOCK), 0, s, jobs, prefix, n, counters);
    return hipGetLastError();
}

}  // namespace

int launch_render_jobs(const dot_render_job* jobs, int n_jobs, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t need = jobs_workspace_bytes(n_jobs);
    if (ws_bytes < need) return fail(DOT_EINVAL, "dot_render_jobs: workspace too small");
    int count[JOB_KINDS] = {};
    for (int i = 0; i < n_jobs; ++i) {
        const dot_render_job& q = jobs[i];
        if (!q.tree || !q.cam || !q.rgb_out) return fail(DOT_EINVAL, "dot_render_jobs: job with a NULL tree, camera or output");
        if (q.width <= 0 || q.height <= 0) return fail(DOT_EINVAL, "dot_render_jobs: job with a non-positive size");
        int64_t nt = (int64_t)((q.width + 7) / 8) * ((q.height + 7) / 8);
        if (q.tile_begin < 0 || q.tile_count < 0 || q.tile_begin + q.tile_count > nt)
            return fail(DOT_EINVAL, "dot_render_jobs: tile range outside the image");
        if (!(q.t_stop >= 0.f && q.t_stop < 1.f)) return fail(DOT_EINVAL, "dot_render_jobs: t_stop must be in [0, 1)");
        ++count[q.tree->storage];
    }
    // host image of the workspace
    std::vector<unsigned char> host(need, 0);
    const size_t prefix_off = sizeof(unsigned long long) * JOB_KINDS * JOB_CHUNKS * CTR_STRIDE;
    int64_t* prefix = reinterpret_cast<int64_t*>(host.data() + prefix_off);
    const size_t jobs_off = (prefix_off + sizeof(int64_t) * (size_t)(n_jobs + JOB_KINDS) + 255) & ~(size_t)255;
    JobDev* jd = reinterpret_cast<JobDev*>(host.data() + jobs_off);
    int first[JOB_KINDS], pfirst[JOB_KINDS], fill[JOB_KINDS];
    int64_t tiles[JOB_KINDS] = {};
    for (int k = 0, jn = 0, pn = 0; k < JOB_KINDS; ++k) {
        first[k] = jn;
        pfirst[k] = pn;
        fill[k] = 0;
        jn += count[k];
        pn += count[k] + 1;
    }
    for (int i = 0; i < n_jobs; ++i) {
        const dot_render_job& q = jobs[i];
        const int k = q.tree->storage;
        const int at = fill[k]++;
        prefix[pfirst[k] + at] = tiles[k];
        tiles[k] += q.tile_count;
        JobDev& d = jd[first[k] + at];
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
    int64_t total = 0;
    for (int k = 0; k < JOB_KINDS; ++k) {
        prefix[pfirst[k] + count[k]] = tiles[k];
        total += tiles[k];
    }
    if (total == 0) return DOT_OK;
    int rc = stage_upload(host.data(), need, ws, s);
    if (rc) return rc;
    unsigned char* base = static_cast<unsigned char*>(ws);
    for (int k = 0; k < JOB_KINDS; ++k) {
        if (tiles[k] == 0) continue;
        const JobDev* jk = reinterpret_cast<const JobDev*>(base + jobs_off) + first[k];
        const int64_t* pk = reinterpret_cast<const int64_t*>(base + prefix_off) + pfirst[k];
        unsigned long long* ck = reinterpret_cast<unsigned long long*>(base) + (size_t)k * JOB_CHUNKS * CTR_STRIDE;
        hipError_t e;
        switch (k) {
            case DOT_F32: e = launch_kind<DOT_F32>(jk, pk, count[k], tiles[k], ck, s); break;
            case DOT_F16: e = launch_kind<DOT_F16>(jk, pk, count[k], tiles[k], ck, s); break;
            case DOT_BF16: e = launch_kind<DOT_BF16>(jk, pk, count[k], tiles[k], ck, s); break;
            default: e = launch_kind<DOT_PAL16>(jk, pk, count[k], tiles[k], ck, s); break;
        }
        if (e != hipSuccess) return hip_fail(e, "dot_render_jobs: launch");
    }
    return DOT_OK;
}

}  // namespace dot
