// Persistent serving queue: one launch that stays resident and renders the
// jobs the host appends while it runs.
//
// Host -> device: jobs are written into a ring of records in pinned,
// host-coherent memory and published by a counter.  One wave of the launch
// (workgroup 0, wave 0: the "feeder") polls that counter, copies each newly
// published job into a device job table and schedules its work items into
// the tile rings, one ring per XCD, each receiving a contiguous eighth of the
// job's tiles, a share at a time beside the other jobs in flight.  An item is
// a run of up to kMaxRun consecutive 8x8 tiles of one job (job slot, first
// tile index in the image, run length in one 64-bit entry); the feeder
// advances the rings' published item counts `tail`.
//
// Workers (every other workgroup): a wave claims the next item of its XCD's
// ring with an atomic on that ring's `next`, waits until the feeder has
// published it (or the queue is stopped), reads the item and its job, renders
// the run's tiles with the same per-ray code as dot_render, and counts them
// done for the job; the wave that completes a job's last tile writes the
// job's number + 1 into the job's completion word in host memory.
//
// Publication without L2 writebacks: a release at device scope writes back
// the issuing XCD's whole L2, and one per 64-ray tile capped the launch near
// half of what relaunching reaches.  The pixels are instead written with
// device-scope (written-through) stores, and a wave waits for its stores to
// complete before it counts the tiles done; only the job's last tile issues a
// release (system scope, for the host).  Runs of several tiles save claims:
// a job is cut into about four runs per wave of an XCD, eight if it is the
// only job in flight when admitted (a lone job's tail, its last round of runs,
// stays short; under load the longer runs keep claims few).
//
// Polls are device-coherent loads, served beyond the L2; waves that find no
// work back off (up to about 13 us between polls) so that thousands of idle
// waves do not keep one memory channel busy under the waves that render, and
// the stop flag rides in the top bit of each ring's published count so that a
// poll is one load.
//
// Exit: the host sets `stop` when no job will follow; the feeder then copies
// what is left and sets the stop bit of every ring's published count, and a
// worker that finds its claimed entry unpublished with the stop bit set
// leaves.  The feeder also sets it once the launch has run for the queue's
// time limit, and a waiting worker leaves by its own clock after 9/8 of it, so
// every wave leaves whatever the host does.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <cstring>
#include <vector>

#include "dot_device.h"

namespace dot {

namespace {

constexpr int kTileBits = 20;                           // tile index field of an entry
constexpr uint32_t kTileMask = (1u << kTileBits) - 1u;
constexpr int64_t kMaxImageTiles = 1ll << kTileBits;
constexpr int kMaxJobs = 4096;                          // job slot field of an entry (12 bits)
constexpr int kRings = 8;                               // one tile ring per XCD
constexpr uint64_t kRing = 1ull << 18;                  // entries (runs) per ring
constexpr uint64_t kMaxOpenTiles = 1ull << 19;          // tiles of unfinished jobs (all rings)
constexpr int64_t kMaxRun = 8;                          // tiles per ring entry, at most
constexpr int64_t kMinRun = 1;                          // tiles per ring entry, at least
constexpr uint64_t kStopBit = 1ull << 63;               // in a ring's published count: no entry will follow
constexpr int kMaxNaps = 4;                             // idle backoff: up to 4 x 127 x 64 clocks between polls
constexpr int kSlotShift = 40;                          // entry: slot << 40 | run << 20 | first tile

// One job as the workers read it (device job table) and as the host writes it
// (pinned ring); copied word by word by the feeder.
struct ServeJob {
    TreeView tv;
    dot_camera cam;
    float* rgb;
    int64_t tile_begin, tile_count;
    uint64_t seq;
    int32_t width, height, degree, pad;
    float bg[3];
    float thr;
};
static_assert(sizeof(ServeJob) % 4 == 0, "copied as 32-bit words");
constexpr int kJobWords = (int)(sizeof(ServeJob) / 4);

// host-coherent control words (pinned)
struct alignas(128) ServeHostCtl {
    uint64_t published;      // jobs published by the host
    uint32_t stop;           // host: no job will follow
    uint32_t ended;          // device: the feeder left (after stop, or at the time limit)
    uint32_t timed_out;      // device: the time limit was reached
};

// device control words, each on its own 128-byte line
struct alignas(128) Line64 {
    uint64_t v;
};

struct ServeDevice {
    Line64* next;            // [kRings] entries claimed by workers, per ring
    Line64* tail;            // [kRings] entries published to the workers, per ring (| kStopBit at the end)
    uint32_t* done;          // [max_jobs] tiles rendered per job slot
    ServeJob* jobs;          // [max_jobs] job table
    uint64_t* ring;          // [kRings][kRing] run entries
};

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Polling uses relaxed atomic loads (coherent, but without the cache
// invalidation an acquire implies: thousands of waiting waves issuing
// acquires would keep the L2 invalidating); the data a changed word publishes
// is then read with relaxed atomic loads too, so no wave ever needs an
// acquire.  The feeder publishes entries behind one release fence per round;
// workers count runs after their device-scope stores complete, and only a
// job's last run issues a release (system scope, for the host).
__device__ __forceinline__ uint64_t poll_sys(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t poll_sys32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t poll_dev(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// exclusive prefix sum over the wave's lanes, and the wave's total
__device__ __forceinline__ int64_t wave_excl_sum(int64_t v, int lane, int64_t& total) {
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int64_t y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    total = readlane64(x, WAVE - 1);
    return x - v;
}

// tiles of chunk x of a job of `count` tiles cut into chunks of `chunk`
__device__ __forceinline__ int64_t chunk_len(int64_t count, int64_t chunk, int x) {
    const int64_t a = (int64_t)x * chunk;
    return a >= count ? 0 : (count - a < chunk ? count - a : chunk);
}

// The feeder: one wave, and a scheduler.  Each lane holds one job being
// published (up to 64 at once, admitted in order); the job's tiles are cut
// into kRings contiguous chunks, chunk x going to the ring of XCD
// (job number + x) mod kRings, so every XCD renders a contiguous part of every
// image (its L2 then holds neighbouring tiles), and each chunk into runs of
// `run` tiles.  A ring is topped up only when fewer entries wait in it than
// the XCD has waves, to twice that.  Jobs with few entries left for the ring
// (at most one per wave of the XCD) get all of them first, and the rest of the
// room goes to the larger jobs in admission order: a small request that
// arrives behind a large one starts after about two rounds of entries instead
// of after the whole large image, and two large ones finish one after the
// other instead of both late.
// `cur` (LDS, [64][kRings]): tiles of each of the lane's chunks published.
__device__ void feeder(ServeHostCtl* ctl, const ServeJob* hjobs, const ServeDevice& dv, int max_jobs,
                       uint64_t t0, uint64_t limit_ticks, int64_t workers, int* cur_lds) {
    const int lane = threadIdx.x & (WAVE - 1);
    int* cur = cur_lds + lane * kRings;
    const int64_t ring_waves = workers / kRings > 0 ? workers / kRings : 1;
    const int64_t low = ring_waves, high = 2 * ring_waves;
    uint64_t copied = 0;
    uint64_t tail[kRings] = {};
    int slot = -1, ring0 = 0;              // this lane's job (slot < 0: none)
    uint64_t seq = 0;                      // its admission number
    int64_t begin = 0, count = 0, chunk = 0, run = 1;
    for (;;) {
        const bool late = wall_clock64() - t0 > limit_ticks;
        bool moved = false;
        // admit published jobs while a lane is free: copy the record into the
        // device table, and the free lane takes the job
        const uint64_t pub = uniform64(poll_sys(&ctl->published));
        while (copied < pub && !late) {
            const uint64_t free_lanes = __ballot(slot < 0);
            if (free_lanes == 0) break;
            const int fl = __ffsll((unsigned long long)free_lanes) - 1;
            const bool alone = __popcll(~free_lanes) == 0;     // no other job in flight
            const int js = (int)(copied % (uint64_t)max_jobs);
            const uint32_t* src = reinterpret_cast<const uint32_t*>(hjobs + js);
            uint32_t* dst = reinterpret_cast<uint32_t*>(dv.jobs + js);
            for (int w = lane; w < kJobWords; w += WAVE)
                __hip_atomic_store(dst + w, __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t b0 = (int64_t)uniform64(poll_sys(reinterpret_cast<const uint64_t*>(&hjobs[js].tile_begin)));
            int64_t c0 = (int64_t)uniform64(poll_sys(reinterpret_cast<const uint64_t*>(&hjobs[js].tile_count)));
            // the host validated the range; a record read wrong must still not run away
            c0 = c0 < 0 ? 0 : (c0 > kMaxImageTiles ? kMaxImageTiles : c0);
            if (lane == fl) {
                slot = js;
                seq = copied;
                ring0 = (int)(copied % kRings);
                begin = b0;
                count = c0;
                chunk = (c0 + kRings - 1) / kRings;
                // about four runs per wave of the XCD (eight for a job alone in
                // the queue), so that the last round of runs is short
                run = chunk / ((alone ? 8 : 4) * ring_waves);
                run = run < kMinRun ? kMinRun : (run > kMaxRun ? kMaxRun : run);
                for (int x = 0; x < kRings; ++x) cur[x] = 0;
            }
            ++copied;
            moved = true;
        }
        // the claim counters of the 8 rings, read in parallel
        const int64_t nx = lane < kRings ? (int64_t)poll_dev(&dv.next[lane].v) : 0;
#pragma unroll
        for (int r = 0; r < kRings; ++r) {
            int64_t backlog = (int64_t)(tail[r] - (uint64_t)readlane64(nx, r));
            if (backlog >= low) continue;
            const int x = (r - ring0) & (kRings - 1);       // this lane's chunk for ring r
            const int64_t len_x = slot < 0 ? 0 : chunk_len(count, chunk, x);
            int64_t done_x = slot < 0 ? 0 : cur[x];
            const int64_t base = begin + (int64_t)x * chunk;
            for (int round = 0; round < 4 && backlog < high; ++round) {
                const int64_t left = (len_x - done_x + run - 1) / run;     // entries this lane still has
                const uint64_t act = __ballot(left > 0);
                if (act == 0) break;
                // jobs with at most a wave's worth of entries per wave of the XCD left for
                // this ring take all of them first; the rest of the room goes to the other
                // jobs in admission order (the oldest first, as far as it reaches)
                const int64_t room = high - backlog;
                const bool small = left > 0 && left <= ring_waves;
                int64_t small_total = 0;
                const int64_t small_before = wave_excl_sum(small ? left : 0, lane, small_total);
                int64_t older = 0;          // entries of the large jobs admitted before this one
                for (uint64_t m = __ballot(left > 0 && !small); m; m &= m - 1) {
                    const int j = __ffsll((unsigned long long)m) - 1;
                    if ((uint64_t)readlane64((int64_t)seq, j) < seq) older += readlane64(left, j);
                }
                int64_t n = small ? room - small_before : room - small_total - older;
                n = n < 0 ? 0 : (n > left ? left : n);
                int64_t total = 0;
                const int64_t off = wave_excl_sum(n, lane, total);
                // the entries of each job in turn, written by the whole wave
                uint64_t* ring = dv.ring + (uint64_t)r * kRing;
                for (uint64_t m = act; m; m &= m - 1) {
                    const int j = __ffsll((unsigned long long)m) - 1;
                    const int64_t nj = readlane64(n, j), oj = readlane64(off, j), dj = readlane64(done_x, j);
                    const int64_t lj = readlane64(len_x, j), bj = readlane64(base, j), rj = readlane64(run, j);
                    const uint64_t sj = (uint64_t)__builtin_amdgcn_readlane(slot, j);
                    for (int64_t i = lane; i < nj; i += WAVE) {
                        const int64_t f = dj + i * rj;
                        const int64_t len = lj - f < rj ? lj - f : rj;
                        const uint64_t e = (sj << kSlotShift) | ((uint64_t)len << kTileBits) | ((uint64_t)(bj + f) & kTileMask);
                        __hip_atomic_store(&ring[(tail[r] + (uint64_t)(oj + i)) & (kRing - 1)], e, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                done_x += n * run;
                if (done_x > len_x) done_x = len_x;
                tail[r] += (uint64_t)total;
                backlog += total;
                moved = true;
            }
            if (slot >= 0) cur[x] = (int)done_x;
        }
        // a lane whose job is published in full is free for the next one
        if (slot >= 0) {
            bool all = true;
            for (int x = 0; x < kRings; ++x) all = all && cur[x] >= chunk_len(count, chunk, x);
            if (all) slot = -1;
        }
        if (moved) {
            // the job records and entries before the counts that cover them:
            // one release fence, then the eight counts
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                for (int r = 0; r < kRings; ++r)
                    __hip_atomic_store(&dv.tail[r].v, tail[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const bool stop = __builtin_amdgcn_readfirstlane(poll_sys32(&ctl->stop)) != 0u;
        const bool drained = __ballot(slot >= 0) == 0 && copied == uniform64(poll_sys(&ctl->published));
        if ((stop && drained) || late) {
            if (lane == 0) {
                for (int r = 0; r < kRings; ++r)
                    __hip_atomic_store(&dv.tail[r].v, tail[r] | kStopBit, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                if (late) __hip_atomic_store(&ctl->timed_out, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&ctl->ended, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            return;
        }
        if (!moved) __builtin_amdgcn_s_sleep(32);
    }
}

// a job record read word by word with relaxed coherent loads into
// wave-uniform registers
__device__ __forceinline__ ServeJob read_job(const ServeJob* p) {
    union {
        ServeJob j;
        uint32_t w[kJobWords];
    } u;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int w = 0; w < kJobWords; ++w)
        u.w[w] = __builtin_amdgcn_readfirstlane(__hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    return u.j;
}

template <int DT, int DEG>
__device__ __forceinline__ void serve_tile(const ServeJob& j, int64_t t, int lane, int* stk) {
    const int tw = (j.width + 7) >> 3;
    const int ty = (int)(t / tw), tx = (int)(t - (int64_t)ty * tw);
    const int u = tx * 8 + (lane & 7), v = ty * 8 + (lane >> 3);
    if (u >= j.width || v >= j.height) return;
    Ray r = camera_ray(j.cam, u, v);
    FwdArgs a{};
    a.thr = j.thr;
    FwdSeg<DT, DEG> seg(j.tv, a);
    sh_basis<DEG>((float)r.dx, (float)r.dy, (float)r.dz, seg.Y);
    int desc = 0;
    traverse(j.tv, r, stk, seg, desc);
    // device-scope stores: written through to where every XCD (and a copy
    // engine) sees them, so completing them is all the publication needs
    float* o = j.rgb + 3 * ((int64_t)v * j.width + u);
#pragma unroll
    for (int c = 0; c < 3; ++c)
        __hip_atomic_store(o + c, fmaf(seg.T, j.bg[c], seg.C[c]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DT>
__global__ __launch_bounds__(BLOCK) void serve_loop_kernel(ServeHostCtl* ctl, const ServeJob* hjobs, uint64_t* hdone,
                                                           ServeDevice dv, int max_jobs, uint64_t limit_ticks) {
    __shared__ int stack_lds[LAT * BLOCK];   // the walk's ancestor stacks; the feeder's chunk cursors
    static_assert(LAT * BLOCK >= WAVE * kRings, "feeder cursors fit in the stack array");
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const uint64_t t0 = wall_clock64();
    if (blockIdx.x == 0) {
        if ((tid >> 6) == 0)
            feeder(ctl, hjobs, dv, max_jobs, t0, limit_ticks, (int64_t)(gridDim.x - 1) * (BLOCK / WAVE), stack_lds);
        return;
    }
    // workgroups are dispatched round-robin over the XCDs: this one takes its
    // tiles from its XCD's ring
    const int x = (int)(blockIdx.x % kRings);
    uint64_t* const ring = dv.ring + (uint64_t)x * kRing;
    // the run being rendered: job slot, next tile, tiles left, run length
    int slot = 0;
    int64_t tile = 0, left = 0, len = 0;
    for (;;) {
        if (left == 0) {
            uint64_t t = 0;
            if (lane == 0) t = atomicAdd(reinterpret_cast<unsigned long long*>(&dv.next[x].v), 1ull);
            t = uniform64(t);
            // wait until the feeder has published entry t of this ring; leave on
            // the stop bit, or by this wave's own clock past the time limit (so
            // the launch ends even if the feeder could not set the bit)
            for (int naps = 1;; naps = naps < kMaxNaps ? naps + 1 : kMaxNaps) {
                const uint64_t v = uniform64(poll_dev(&dv.tail[x].v));
                if (t < (v & ~kStopBit)) break;
                if (v & kStopBit) return;
                if (wall_clock64() - t0 > limit_ticks + limit_ticks / 8) return;
                for (int k = 0; k < naps; ++k) __builtin_amdgcn_s_sleep(127);
            }
            // the entry and the job record are read only after the count that
            // published them was seen (their loads are coherent, so no cache
            // needs invalidating; this keeps the compiler from moving them earlier)
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            const uint64_t e = uniform64(__hip_atomic_load(&ring[t & (kRing - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            slot = (int)(e >> kSlotShift);
            tile = (int64_t)(e & kTileMask);
            len = (int64_t)((e >> kTileBits) & kTileMask);
            // cannot happen for a published entry; never index past the table
            if (slot >= max_jobs || len < 1 || len > kMaxRun) continue;
            left = len;
        }
        // the job record is read again for every tile: kept in registers across
        // the run it would raise the kernel's register count and cut occupancy
        const ServeJob j = read_job(dv.jobs + slot);
        switch (j.degree) {
            case 0: serve_tile<DT, 0>(j, tile, lane, &stack_lds[tid]); break;
            case 1: serve_tile<DT, 1>(j, tile, lane, &stack_lds[tid]); break;
            case 2: serve_tile<DT, 2>(j, tile, lane, &stack_lds[tid]); break;
            default: serve_tile<DT, 3>(j, tile, lane, &stack_lds[tid]); break;
        }
        ++tile;
        if (--left > 0) continue;
        // the run's pixels before its count: they are device-coherent stores,
        // so waiting for this wave's stores to complete orders them before the
        // count (a release here would also write back the XCD's whole L2,
        // which bounded the launch); the job's last tile publishes the job to
        // the host with a system-scope release
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0) {
            const uint32_t c = __hip_atomic_fetch_add(&dv.done[slot], (uint32_t)len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + (uint32_t)len;
            if ((int64_t)c == j.tile_count) {
                __hip_atomic_store(&dv.done[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __atomic_thread_fence(__ATOMIC_SEQ_CST);
                __hip_atomic_store(&hdone[slot], j.seq + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

__global__ void zero_words(uint32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// workers: all the workgroups the CUs hold but one per CU, which stays free so
// that other launches (copies, other streams' kernels) still find room while
// the queue is open
template <int DT>
int resident_grid() {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, serve_loop_kernel<DT>, BLOCK, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 2;
        cus = 256;
    }
    return (per_cu > 1 ? per_cu - 1 : 1) * cus;
}

}  // namespace

}  // namespace dot

struct dot_serve_queue {
    int storage = 0, max_jobs = 0;
    double max_seconds = 0.0;
    hipStream_t stream = nullptr;
    hipEvent_t ended = nullptr;
    dot::ServeHostCtl* ctl = nullptr;       // pinned
    dot::ServeJob* hjobs = nullptr;         // pinned [max_jobs]
    uint64_t* hdone = nullptr;              // pinned [max_jobs]
    void* dmem = nullptr;                   // device: control lines, done, jobs, ring
    dot::ServeDevice dv{};
    uint64_t pushed = 0, oldest = 0, open_tiles = 0;
    std::vector<int64_t> tiles_of;          // tiles of the job in each slot
};

namespace dot {
namespace {

void free_queue(dot_serve_queue* q) {
    if (q->ended) (void)hipEventDestroy(q->ended);
    if (q->dmem) (void)hipFree(q->dmem);
    if (q->ctl) (void)hipHostFree(q->ctl);
    if (q->hjobs) (void)hipHostFree(q->hjobs);
    if (q->hdone) (void)hipHostFree(q->hdone);
    delete q;
}

// retire jobs completed in order from the oldest unfinished one
void retire(dot_serve_queue* q) {
    while (q->oldest < q->pushed) {
        const int slot = (int)(q->oldest % (uint64_t)q->max_jobs);
        const uint64_t w = __atomic_load_n(&q->hdone[slot], __ATOMIC_ACQUIRE);
        if (w != q->oldest + 1) break;
        q->open_tiles -= (uint64_t)q->tiles_of[slot];
        ++q->oldest;
    }
}

bool launch_ended(dot_serve_queue* q) { return __atomic_load_n(&q->ctl->ended, __ATOMIC_ACQUIRE) != 0u; }

}  // namespace
}  // namespace dot

extern "C" {

int dot_serve_open(int32_t storage, int32_t max_jobs, double max_seconds, void* stream, dot_serve_t* out) {
    using namespace dot;
    if (!out) return fail(DOT_EINVAL, "dot_serve_open: out is NULL");
    *out = nullptr;
    if (storage < DOT_F32 || storage > DOT_PAL16) return fail(DOT_EINVAL, "dot_serve_open: unknown storage type");
    if (max_jobs < 1 || max_jobs > kMaxJobs) return fail(DOT_EINVAL, "dot_serve_open: max_jobs must be in 1..4096");
    if (!(max_seconds > 0.0) || !std::isfinite(max_seconds))
        return fail(DOT_EINVAL, "dot_serve_open: max_seconds must be positive and finite");
    auto* q = new (std::nothrow) dot_serve_queue();
    if (!q) return fail(DOT_ENOMEM, "dot_serve_open: out of host memory");
    q->storage = storage;
    q->max_jobs = max_jobs;
    q->max_seconds = max_seconds;
    q->stream = static_cast<hipStream_t>(stream);
    q->tiles_of.assign((size_t)max_jobs, 0);
    hipError_t e = hipHostMalloc((void**)&q->ctl, sizeof(ServeHostCtl), hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void**)&q->hjobs, sizeof(ServeJob) * (size_t)max_jobs, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void**)&q->hdone, sizeof(uint64_t) * (size_t)max_jobs, hipHostMallocCoherent);
    const size_t lines = 2 * kRings * sizeof(Line64);
    const size_t done_b = ((sizeof(uint32_t) * (size_t)max_jobs) + 255) & ~(size_t)255;
    const size_t jobs_b = ((sizeof(ServeJob) * (size_t)max_jobs) + 255) & ~(size_t)255;
    const size_t total = lines + done_b + jobs_b + sizeof(uint64_t) * kRing * kRings;
    if (e == hipSuccess) e = hipMalloc(&q->dmem, total);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ended, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_queue(q);
        return hip_fail(e, "dot_serve_open: allocation");
    }
    std::memset(q->ctl, 0, sizeof(ServeHostCtl));
    std::memset(q->hjobs, 0, sizeof(ServeJob) * (size_t)max_jobs);
    std::memset(q->hdone, 0, sizeof(uint64_t) * (size_t)max_jobs);
    char* base = static_cast<char*>(q->dmem);
    q->dv.next = reinterpret_cast<Line64*>(base);
    q->dv.tail = q->dv.next + kRings;
    q->dv.done = reinterpret_cast<uint32_t*>(base + lines);
    q->dv.jobs = reinterpret_cast<ServeJob*>(base + lines + done_b);
    q->dv.ring = reinterpret_cast<uint64_t*>(base + lines + done_b + jobs_b);
    int dev = 0, khz = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess && khz <= 0) e = hipErrorInvalidValue;
    if (e != hipSuccess) {
        free_queue(q);
        return hip_fail(e, "dot_serve_open: wall clock rate");
    }
    const double ticks = max_seconds * (double)khz * 1e3;
    const uint64_t limit = ticks >= 1.8e19 ? ~0ull : (uint64_t)ticks;
    // the control lines, completion counts and job table start at zero (a kernel, not a memset)
    const int64_t zwords = (int64_t)((lines + done_b + jobs_b) / 4);
    hipLaunchKernelGGL(zero_words, dim3(256), dim3(256), 0, q->stream, reinterpret_cast<uint32_t*>(q->dmem), zwords);
    int grid = 0;
    switch (storage) {
        case DOT_F32: grid = resident_grid<DOT_F32>(); break;
        case DOT_F16: grid = resident_grid<DOT_F16>(); break;
        case DOT_BF16: grid = resident_grid<DOT_BF16>(); break;
        default: grid = resident_grid<DOT_PAL16>(); break;
    }
    const dim3 g((unsigned)(grid + 1)), b(BLOCK);
    switch (storage) {
        case DOT_F32: hipLaunchKernelGGL(serve_loop_kernel<DOT_F32>, g, b, 0, q->stream, q->ctl, q->hjobs, q->hdone, q->dv, max_jobs, limit); break;
        case DOT_F16: hipLaunchKernelGGL(serve_loop_kernel<DOT_F16>, g, b, 0, q->stream, q->ctl, q->hjobs, q->hdone, q->dv, max_jobs, limit); break;
        case DOT_BF16: hipLaunchKernelGGL(serve_loop_kernel<DOT_BF16>, g, b, 0, q->stream, q->ctl, q->hjobs, q->hdone, q->dv, max_jobs, limit); break;
        default: hipLaunchKernelGGL(serve_loop_kernel<DOT_PAL16>, g, b, 0, q->stream, q->ctl, q->hjobs, q->hdone, q->dv, max_jobs, limit); break;
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(q->ended, q->stream);
    if (e != hipSuccess) {
        // nothing may still run on the queue's memory: stop a launch that did start, then wait for it
        __atomic_store_n(&q->ctl->stop, 1u, __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(q->stream);
        free_queue(q);
        return hip_fail(e, "dot_serve_open: launch");
    }
    *out = q;
    return DOT_OK;
}

int dot_serve_push(dot_serve_t q, const dot_serve_job* job, int64_t* ticket) {
    using namespace dot;
    if (!q || !job || !ticket) return fail(DOT_EINVAL, "dot_serve_push: NULL argument");
    if (!job->tree || !job->rgb_out) return fail(DOT_EINVAL, "dot_serve_push: job with a NULL tree or output");
    if (job->tree->storage != q->storage)
        return fail(DOT_EINVAL, "dot_serve_push: the tree's storage type is not the queue's");
    if (job->width <= 0 || job->height <= 0) return fail(DOT_EINVAL, "dot_serve_push: non-positive image size");
    const int64_t nt = (int64_t)((job->width + 7) / 8) * ((job->height + 7) / 8);
    if (nt > kMaxImageTiles) return fail(DOT_EINVAL, "dot_serve_push: image of more than 2^20 tiles");
    if (job->tile_begin < 0 || job->tile_count < 1 || job->tile_begin + job->tile_count > nt)
        return fail(DOT_EINVAL, "dot_serve_push: tile range outside the image");
    if (!(job->t_stop >= 0.f && job->t_stop < 1.f)) return fail(DOT_EINVAL, "dot_serve_push: t_stop must be in [0, 1)");
    if (launch_ended(q)) return fail(DOT_EHIP, "dot_serve_push: the queue's launch has ended");
    retire(q);
    if (q->pushed - q->oldest >= (uint64_t)q->max_jobs || q->open_tiles + (uint64_t)job->tile_count > kMaxOpenTiles)
        return fail(DOT_EBUSY, "dot_serve_push: queue full");
    const int slot = (int)(q->pushed % (uint64_t)q->max_jobs);
    ServeJob& r = q->hjobs[slot];
    r.tv = job->tree->view();
    r.cam = job->cam;
    r.rgb = job->rgb_out;
    r.tile_begin = job->tile_begin;
    r.tile_count = job->tile_count;
    r.seq = q->pushed;
    r.width = job->width;
    r.height = job->height;
    r.degree = job->tree->degree;
    r.pad = 0;
    for (int a = 0; a < 3; ++a) r.bg[a] = job->bg[a];
    r.thr = job->t_stop > 0.f ? -std::log(job->t_stop) : __builtin_huge_valf();
    q->tiles_of[slot] = job->tile_count;
    q->open_tiles += (uint64_t)job->tile_count;
    *ticket = (int64_t)q->pushed;
    ++q->pushed;
    // the record before the count that publishes it
    __atomic_store_n(&q->ctl->published, q->pushed, __ATOMIC_RELEASE);
    return DOT_OK;
}

int dot_serve_done(dot_serve_t q, int64_t ticket) {
    using namespace dot;
    if (!q) return fail(DOT_EINVAL, "dot_serve_done: NULL queue");
    if (ticket < 0 || (uint64_t)ticket >= q->pushed) return fail(DOT_EINVAL, "dot_serve_done: unknown ticket");
    if ((uint64_t)ticket + (uint64_t)q->max_jobs < q->pushed) return 1;   // its slot was reused: it had completed
    const int slot = (int)((uint64_t)ticket % (uint64_t)q->max_jobs);
    if (__atomic_load_n(&q->hdone[slot], __ATOMIC_ACQUIRE) == (uint64_t)ticket + 1) return 1;
    if (launch_ended(q) && __atomic_load_n(&q->hdone[slot], __ATOMIC_ACQUIRE) != (uint64_t)ticket + 1) {
        // the launch may have ended with the job's last tile still being written: wait for the kernel
        if (hipEventQuery(q->ended) == hipSuccess && __atomic_load_n(&q->hdone[slot], __ATOMIC_ACQUIRE) != (uint64_t)ticket + 1)
            return fail(DOT_EHIP, "dot_serve_done: the queue's launch ended before the job completed");
    }
    return 0;
}

int dot_serve_close(dot_serve_t q) {
    using namespace dot;
    if (!q) return DOT_OK;
    __atomic_store_n(&q->ctl->stop, 1u, __ATOMIC_RELEASE);
    // the launch ends once it has rendered what was published, and by its own
    // clock within 9/8 of its time limit whatever happens; wait that long
    // (plus a margin) and never block beyond it
    const auto t0 = std::chrono::steady_clock::now();
    const double limit = q->max_seconds * 1.25 + 10.0;
    for (;;) {
        const hipError_t e = hipEventQuery(q->ended);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) return hip_fail(e, "dot_serve_close: waiting for the launch");
        if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit)
            return fail(DOT_EHIP, "dot_serve_close: the launch did not end (the queue is left allocated)");
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    free_queue(q);
    return DOT_OK;
}

}  // extern "C"
