// Forward renderer (Eq. 1-2 with the fused training signal) and its adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dot_device.h"

namespace dot {

// MODE 0: plain; 1: with the traversal counters of dot_render_stats; 2: with
// the per-leaf segment counts of a training forward
template <int DT, int DEG, int MODE>
__global__ __launch_bounds__(BLOCK) void render_fwd_kernel(TreeView tv, RayBatch rb, FwdArgs a) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t nb = gridDim.x;
    const int64_t tile = xcd_block(blockIdx.x, nb) * WAVES_PER_BLOCK + (tid >> 6);
    if (tile >= rb.n_tiles) return;
    Ray r;
    int64_t rid;
    if (!make_ray(rb, tile, lane, r, rid)) return;
    FwdSeg<DT, DEG, MODE == 2> seg(tv, a);
    seg.rid = rid;
    sh_basis<DEG>((float)r.dx, (float)r.dy, (float)r.dz, seg.Y);
    int desc = 0;
    traverse(tv, r, &stack_lds[tid], seg, desc);
    if constexpr (MODE == 2) {
        if (a.rec.a) {
            seg.flush_slot();
            a.rec.count[rid] = seg.nrec;
            if (seg.nrec > a.rec.cap) a.rec.olist[atomicAdd(a.rec.overflow, 1u)] = (int32_t)rid;
            // every segment counted above is one bucket row (one atomic per wave
            // after the compiler's wave reduction of a same-address add)
            atomicAdd(a.rec.total, (uint32_t)seg.nrec);
        }
    }
    if (a.rgb) {
        float Te = seg.T;
        a.rgb[3 * rid + 0] = fmaf(Te, a.bg[0], seg.C[0]);
        a.rgb[3 * rid + 1] = fmaf(Te, a.bg[1], seg.C[1]);
        a.rgb[3 * rid + 2] = fmaf(Te, a.bg[2], seg.C[2]);
    }
    if (a.nseg) a.nseg[rid] = seg.n;
    if constexpr (MODE == 1) {
        atomicAdd(&a.stats[0], 1ull);
        atomicAdd(&a.stats[1], (unsigned long long)seg.n);
        atomicAdd(&a.stats[2], (unsigned long long)seg.fetched);
        atomicAdd(&a.stats[3], (unsigned long long)desc);
    }
}

// Adjoint: replay the forward segments and push dL/dsigma, dL/dsh.
template <int DT, int DEG>
struct BwdSeg {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    const TreeView& tv;
    const BwdArgs& a;
    float Y[K];
    float S = 0.f, T = 1.f;
    float C[3], g[3];
    float P[3] = {0.f, 0.f, 0.f};
    int n = 0, limit = 0;

    __device__ BwdSeg(const TreeView& tv_, const BwdArgs& a_) : tv(tv_), a(a_) {}

    __device__ __forceinline__ bool operator()(int leaf, float delta) {
        ++n;
        // dC/dsigma = delta (T_{i+1} c - (C - P_i)) is non-zero for any sigma > 0,
        // even when sigma * delta underflows, so the leaf colour is always needed
        float sraw = load_sigma<DT>(tv.sigma, leaf);
        if (sraw > 0.f) {
            float tau = sraw * delta;
            float Sn = S + tau;
            float Tn = __expf(-Sn);
            float w = fmaxf(T - Tn, 0.f);
            float row[3 * K];
            load_sh_row<DT, 3 * K>(tv.sh, leaf, row);
            float c[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float x = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) x = fmaf(row[ch * K + k], Y[k], x);
                c[ch] = sigmoidf_(x);
            }
            float gs = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                P[ch] = fmaf(w, c[ch], P[ch]);
                gs = fmaf(g[ch], Tn * c[ch] - (C[ch] - P[ch]), gs);
            }
            unsafeAtomicAdd(&a.grad_sigma[leaf], gs * delta);
            if (w > 0.f) {
                float* gh = a.grad_sh + (int64_t)leaf * (3 * K);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    float f = g[ch] * w * c[ch] * (1.f - c[ch]);
#pragma unroll
                    for (int k = 0; k < K; ++k) unsafeAtomicAdd(&gh[ch * K + k], f * Y[k]);
                }
            }
            S = Sn;
            T = Tn;
        }
        return n < limit;
    }
};

template <int DT, int DEG>
__global__ __launch_bounds__(BLOCK) void render_bwd_kernel(TreeView tv, RayBatch rb, BwdArgs a) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t nb = gridDim.x;
    const int64_t tile = xcd_block(blockIdx.x, nb) * WAVES_PER_BLOCK + (tid >> 6);
    if (tile >= rb.n_tiles) return;
    Ray r;
    int64_t rid;
    if (!make_ray(rb, tile, lane, r, rid)) return;
    BwdSeg<DT, DEG> seg(tv, a);
    seg.limit = a.nseg[rid];
    if (seg.limit <= 0) return;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        seg.C[ch] = a.rgb_fwd[3 * rid + ch];
        seg.g[ch] = a.grad_rgb[3 * rid + ch];
    }
    if (seg.g[0] == 0.f && seg.g[1] == 0.f && seg.g[2] == 0.f) return;
    sh_basis<DEG>((float)r.dx, (float)r.dy, (float)r.dz, seg.Y);
    int desc = 0;
    traverse(tv, r, &stack_lds[tid], seg, desc);
}

// ---------------------------------------------------------------------------
// Re-traversal adjoint with the lanes' terms summed per leaf inside the
// wavefront before the float atomics.  At a traversal step the lanes that
// composite a segment form runs of equal leaf id in lane order (neighbouring
// pixels of a tile often cross the same leaf); a segmented reduction over
// those runs (a Hillis-Steele scan toward each run's first lane, lane
// shuffles over distances 1, 2, 4, ..., stopped at the first distance with no
// partner) leaves each run's sum in its first lane, which alone issues the
// 1 + 3K atomics (the SH terms one channel of K at a time).  Inactive lanes (finished rays, zero-length steps) and
// segments with sigma <= 0 never join a run.  No scratch and no host
// synchronisation.
// ---------------------------------------------------------------------------
// Sums v over the runs of equal key among the lanes calling it and leaves each
// run's sum in its first lane; returns true in those lanes (key >= 0).
template <int NV>
__device__ __forceinline__ bool leaf_runs_sum(int key, float (&v)[NV]) {
    const int lane = (int)__lane_id();
    const uint64_t act = __ballot(1);
    const int prev = __shfl_up(key, 1);
    const bool prev_in = lane > 0 && ((act >> (lane - 1)) & 1ull) && prev == key;
    const uint64_t heads = __ballot(!prev_in);
    if (heads != act) {
        // run number of each lane: the heads at or below it
        const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const int run = __popcll(heads & le);
        for (int s = 1; s < WAVE; s <<= 1) {
            const int r2 = __shfl_down(run, s);
            const bool ok = lane + s < WAVE && ((act >> (lane + s)) & 1ull) && r2 == run;
            if (!__any(ok)) break;      // runs are contiguous: no partner at s, none farther
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const float w = __shfl_down(v[j], s);
                if (ok) v[j] += w;
            }
        }
    }
    return !prev_in && key >= 0;
}

template <int DT, int DEG>
struct BwdSegWave {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    const TreeView& tv;
    const BwdArgs& a;
    float Y[K];
    float S = 0.f, T = 1.f;
    float C[3], g[3];
    float P[3] = {0.f, 0.f, 0.f};
    int n = 0, limit = 0;

    __device__ BwdSegWave(const TreeView& tv_, const BwdArgs& a_) : tv(tv_), a(a_) {}

    __device__ __forceinline__ bool operator()(int leaf, float delta) {
        ++n;
        const float sraw = load_sigma<DT>(tv.sigma, leaf);
        // per lane: the density term and the SH factors f_ch (the SH terms are
        // f_ch Y_k, formed one channel at a time to keep few values live)
        float d[2] = {0.f, 0.f};        // dL/dsigma, and 1 if any SH term is non-zero
        float f[3] = {0.f, 0.f, 0.f};
        if (sraw > 0.f) {
            const float tau = sraw * delta;
            const float Sn = S + tau;
            const float Tn = __expf(-Sn);
            const float w = fmaxf(T - Tn, 0.f);
            float row[3 * K];
            load_sh_row<DT, 3 * K>(tv.sh, leaf, row);
            float c[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float x = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) x = fmaf(row[ch * K + k], Y[k], x);
                c[ch] = sigmoidf_(x);
            }
            float gs = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                P[ch] = fmaf(w, c[ch], P[ch]);
                gs = fmaf(g[ch], Tn * c[ch] - (C[ch] - P[ch]), gs);
            }
            d[0] = gs * delta;
            if (w > 0.f) {
                d[1] = 1.f;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) f[ch] = g[ch] * w * c[ch] * (1.f - c[ch]);
            }
            S = Sn;
            T = Tn;
        }
        const int key = sraw > 0.f ? leaf : -1;
        const bool head = leaf_runs_sum<2>(key, d);
        if (head) unsafeAtomicAdd(&a.grad_sigma[leaf], d[0]);
        if (__any(head && d[1] > 0.f)) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float v[K];
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] = f[ch] * Y[k];
                leaf_runs_sum<K>(key, v);
                if (head && d[1] > 0.f) {
                    float* gh = a.grad_sh + (int64_t)leaf * (3 * K) + ch * K;
#pragma unroll
                    for (int k = 0; k < K; ++k) unsafeAtomicAdd(&gh[k], v[k]);
                }
            }
        }
        return n < limit;
    }
};

template <int DT, int DEG>
__global__ __launch_bounds__(BLOCK) void render_bwd_wave_kernel(TreeView tv, RayBatch rb, BwdArgs a) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t nb = gridDim.x;
    const int64_t tile = xcd_block(blockIdx.x, nb) * WAVES_PER_BLOCK + (tid >> 6);
    if (tile >= rb.n_tiles) return;
    Ray r;
    int64_t rid;
    if (!make_ray(rb, tile, lane, r, rid)) return;
    BwdSegWave<DT, DEG> seg(tv, a);
    seg.limit = a.nseg[rid];
    if (seg.limit <= 0) return;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        seg.C[ch] = a.rgb_fwd[3 * rid + ch];
        seg.g[ch] = a.grad_rgb[3 * rid + ch];
    }
    if (seg.g[0] == 0.f && seg.g[1] == 0.f && seg.g[2] == 0.f) return;
    sh_basis<DEG>((float)r.dx, (float)r.dy, (float)r.dz, seg.Y);
    int desc = 0;
    traverse(tv, r, &stack_lds[tid], seg, desc);
}

// ---------------------------------------------------------------------------
// Leaf-bucketed adjoint.  Many rays cross the same leaves, so pushing every
// segment's 1 + 3K gradient terms with float atomics serialises on the hot
// leaves.  Instead: (1) count the contributing segments of every leaf, (2)
// scan the counts into bucket offsets, (3) write each segment's gradient row
// into its leaf's bucket, and (4) reduce every bucket into the gradient
// arrays.  A bucket has two regions: the rows of the segments a training
// forward recorded, at the slots the forward reserved (replayed without
// atomics), then the rows of the other segments, whose slots an integer
// atomic on the leaf's cursor picks as they are emitted.  The SH gradient of a
// segment is the outer product a_ch Y_k(d) with a_ch = g_ch w c_ch (1 - c_ch),
// so a row stores dsigma, a[3] and the ray direction (8 floats; 4 at degree 0,
// where Y is constant) and the reduction re-evaluates Y(d) -- 32 B per segment
// instead of (1 + 3K) floats.
// ---------------------------------------------------------------------------
template <int DT>
struct BwdCount {
    const TreeView& tv;
    uint32_t* count;
    int n = 0, limit = 0;
    __device__ BwdCount(const TreeView& tv_, uint32_t* c) : tv(tv_), count(c) {}
    __device__ __forceinline__ bool operator()(int leaf, float delta) {
        ++n;
        if (load_sigma<DT>(tv.sigma, leaf) > 0.f) atomicAdd(&count[leaf], 1u);
        return n < limit;
    }
};

// floats per bucket row: dsigma, a[3], then the direction when Y depends on it
template <int DEG>
constexpr int bwd_row_floats() { return DEG == 0 ? 4 : 8; }
inline int bwd_row_floats_rt(int deg) { return deg == 0 ? 4 : 8; }

// Emits the rows of the segments in the second region of their buckets:
// slot = base0[leaf] (recorded rows, or none) + the cursor's count.  The first
// `skip` contributing segments of the ray (the recorded ones) only advance the
// prefix sums.
template <int DT, int DEG>
struct BwdEmit {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    static constexpr int RS = bwd_row_floats<DEG>();
    const TreeView& tv;
    const uint32_t* offset;
    const uint32_t* base0;    // [L] rows of the recorded region, or null
    const uint32_t* count;    // [L] rows of the second region
    uint32_t* cursor;
    float* rows;
    uint32_t n_rows;          // rows of the bucket array: every store stays below it
    float Y[K];
    float d[3];
    float S = 0.f, T = 1.f;
    float C[3], g[3];
    float P[3] = {0.f, 0.f, 0.f};
    int n = 0, limit = 0;
    int skip = 0;             // contributing segments not to emit

    __device__ BwdEmit(const TreeView& tv_, const uint32_t* o, const uint32_t* b0, const uint32_t* n_, uint32_t* c,
                       float* r, uint32_t nr)
        : tv(tv_), offset(o), base0(b0), count(n_), cursor(c), rows(r), n_rows(nr) {}

    __device__ __forceinline__ bool operator()(int leaf, float delta) {
        ++n;
        float sraw = load_sigma<DT>(tv.sigma, leaf);
        if (sraw > 0.f && skip > 0) {
            // a recorded segment: its row comes from the replay
            --skip;
            const float Sn = S + sraw * delta;
            const float Tn = __expf(-Sn);
            const float w = fmaxf(T - Tn, 0.f);
            float row[3 * K];
            load_sh_row<DT, 3 * K>(tv.sh, leaf, row);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float x = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) x = fmaf(row[ch * K + k], Y[k], x);
                P[ch] = fmaf(w, sigmoidf_(x), P[ch]);
            }
            S = Sn;
            T = Tn;
        } else if (sraw > 0.f) {
            float tau = sraw * delta;
            float Sn = S + tau;
            float Tn = __expf(-Sn);
            float w = fmaxf(T - Tn, 0.f);
            float row[3 * K];
            load_sh_row<DT, 3 * K>(tv.sh, leaf, row);
            float c[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float x = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) x = fmaf(row[ch * K + k], Y[k], x);
                c[ch] = sigmoidf_(x);
            }
            float out[RS];
            float gs = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                P[ch] = fmaf(w, c[ch], P[ch]);
                gs = fmaf(g[ch], Tn * c[ch] - (C[ch] - P[ch]), gs);
            }
            out[0] = gs * delta;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) out[1 + ch] = w > 0.f ? g[ch] * w * c[ch] * (1.f - c[ch]) : 0.f;
            if constexpr (RS == 8) {
                out[4] = d[0];
                out[5] = d[1];
                out[6] = d[2];
                out[7] = 0.f;
            }
            // the region holds exactly the segments the counting found; a slot
            // past it is never written (the reduction reads written rows only)
            uint32_t k = atomicAdd(&cursor[leaf], 1u);
            const uint64_t slot = (uint64_t)offset[leaf] + (base0 ? base0[leaf] : 0u) + k;
            if (k < count[leaf] && slot < n_rows) {
                float4* dst = reinterpret_cast<float4*>(rows + (int64_t)slot * RS);
#pragma unroll
                for (int j = 0; j < RS / 4; ++j)
                    dst[j] = make_float4(out[4 * j], out[4 * j + 1], out[4 * j + 2], out[4 * j + 3]);
            }
            S = Sn;
            T = Tn;
        }
        return n < limit;
    }
};

template <int DT>
__global__ __launch_bounds__(BLOCK) void bwd_count_kernel(TreeView tv, RayBatch rb, BwdArgs a, uint32_t* count) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (tid >> 6);
    if (tile >= rb.n_tiles) return;
    Ray r;
    int64_t rid;
    if (!make_ray(rb, tile, lane, r, rid)) return;
    BwdCount<DT> seg(tv, count);
    seg.limit = a.nseg[rid];
    if (seg.limit <= 0) return;
    if (a.grad_rgb[3 * rid] == 0.f && a.grad_rgb[3 * rid + 1] == 0.f && a.grad_rgb[3 * rid + 2] == 0.f) return;
    int desc = 0;
    traverse(tv, r, &stack_lds[tid], seg, desc);
}

template <int DT, int DEG>
__global__ __launch_bounds__(BLOCK) void bwd_emit_kernel(TreeView tv, RayBatch rb, BwdArgs a, const uint32_t* offset,
                                                         const uint32_t* base0, const uint32_t* count, uint32_t* cursor,
                                                         float* rows) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (tid >> 6);
    if (tile >= rb.n_tiles) return;
    Ray r;
    int64_t rid;
    if (!make_ray(rb, tile, lane, r, rid)) return;
    BwdEmit<DT, DEG> seg(tv, offset, base0, count, cursor, rows, a.n_rows);
    seg.limit = a.nseg[rid];
    if (seg.limit <= 0) return;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        seg.C[ch] = a.rgb_fwd[3 * rid + ch];
        seg.g[ch] = a.grad_rgb[3 * rid + ch];
    }
    if (seg.g[0] == 0.f && seg.g[1] == 0.f && seg.g[2] == 0.f) return;
    seg.d[0] = (float)r.dx;
    seg.d[1] = (float)r.dy;
    seg.d[2] = (float)r.dz;
    sh_basis<DEG>(seg.d[0], seg.d[1], seg.d[2], seg.Y);
    int desc = 0;
    traverse(tv, r, &stack_lds[tid], seg, desc);
}

// Re-traversal of the rays with more segments than the records hold (their
// ids listed by the forward), one ray per lane: the recorded first `cap`
// contributing segments only advance the prefix sums, the rest are emitted.
template <int DT, int DEG>
__global__ __launch_bounds__(BLOCK) void bwd_emit_list_kernel(TreeView tv, RayBatch rb, BwdArgs a, const int32_t* list,
                                                              int64_t nlist, const uint32_t* offset,
                                                              const uint32_t* base0, const uint32_t* count,
                                                              uint32_t* cursor, float* rows) {
    __shared__ int stack_lds[LAT * BLOCK];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + tid;
    if (i >= nlist) return;
    const int64_t rid = list[i];
    if (rid < 0 || rid >= rb.n_rays) return;
    Ray r = ray_of(rb, rid);
    BwdEmit<DT, DEG> seg(tv, offset, base0, count, cursor, rows, a.n_rows);
    seg.limit = a.nseg[rid];
    seg.skip = a.rec.cap;
    if (seg.limit <= 0) return;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        seg.C[ch] = a.rgb_fwd[3 * rid + ch];
        seg.g[ch] = a.grad_rgb[3 * rid + ch];
    }
    if (seg.g[0] == 0.f && seg.g[1] == 0.f && seg.g[2] == 0.f) return;
    seg.d[0] = (float)r.dx;
    seg.d[1] = (float)r.dy;
    seg.d[2] = (float)r.dz;
    sh_basis<DEG>(seg.d[0], seg.d[1], seg.d[2], seg.Y);
    int desc = 0;
    traverse(tv, r, &stack_lds[tid], seg, desc);
}

// Replay of the forward's segment records (of every ray, the first `cap` of
// a ray with more): the same per-segment arithmetic as BwdEmit, without the
// traversal and the leaf fetches, each row stored at the slot the forward
// reserved.  Every record's row is written (zero for a ray with g = 0), since
// the recorded region of a bucket has no cursor.  The next record and its
// leaf's bucket offset are requested one record ahead, so the stores do not
// wait on them.  Same ray-to-lane mapping as the traversal kernels.
template <int DEG>
__global__ __launch_bounds__(BLOCK) void bwd_emit_rec_kernel(RayBatch rb, BwdArgs a, int64_t L, const uint32_t* offset,
                                                             uint32_t n_rows, float* rows) {
    constexpr int RS = bwd_row_floats<DEG>();
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (tid >> 6);
    if (tile >= rb.n_tiles) return;
    Ray r;
    int64_t rid;
    if (!make_ray(rb, tile, lane, r, rid)) return;
    int nrec = a.rec.count[rid];
    if (nrec <= 0) return;
    if (nrec > a.rec.cap) nrec = a.rec.cap;
    float g[3], C[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        C[ch] = a.rgb_fwd[3 * rid + ch];
        g[ch] = a.grad_rgb[3 * rid + ch];
    }
    const float d[3] = {(float)r.dx, (float)r.dy, (float)r.dz};
    float S = 0.f, T = 1.f, P[3] = {0.f, 0.f, 0.f};
    auto load_rec = [&](int i, float4& A_, float2& B_, uint32_t& s_) {
        const int64_t j = (int64_t)i * a.rec.n + rid;
        A_ = a.rec.a[j];
        B_ = a.rec.b[j];
        s_ = a.rec.slot[j];
    };
    // record i (with its bucket offset), record i + 1
    float4 A0, A1;
    float2 B0, B1;
    uint32_t s0 = 0, s1 = 0;
    load_rec(0, A0, B0, s0);
    A1 = A0;
    B1 = B0;
    if (nrec > 1) load_rec(1, A1, B1, s1);
    // A slot is below its leaf's recorded count by construction; records of
    // another batch or tree are caught only as far as staying in bounds goes
    // (leaf id < L, row < n_rows), so the one per-leaf read is the offset.
    int leaf0 = __float_as_int(A0.x);
    bool ok0 = (uint64_t)(uint32_t)leaf0 < (uint64_t)L;
    uint32_t off0 = ok0 ? offset[leaf0] : 0u;
    for (int i = 0; i < nrec && ok0; ++i) {
        // record i + 1's bucket offset and record i + 2 are requested first
        bool ok1 = false;
        uint32_t off1 = 0;
        float4 A2 = A1;
        float2 B2 = B1;
        uint32_t s2 = s1;
        if (i + 1 < nrec) {
            const int leaf1 = __float_as_int(A1.x);
            ok1 = (uint64_t)(uint32_t)leaf1 < (uint64_t)L;
            if (ok1) off1 = offset[leaf1];
            if (i + 2 < nrec) load_rec(i + 2, A2, B2, s2);
        }
        const float delta = A0.y, tau = A0.z;
        const float c[3] = {A0.w, B0.x, B0.y};
        const float Sn = S + tau;
        const float Tn = __expf(-Sn);
        const float w = fmaxf(T - Tn, 0.f);
        float out[RS];
        float gs = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            P[ch] = fmaf(w, c[ch], P[ch]);
            gs = fmaf(g[ch], Tn * c[ch] - (C[ch] - P[ch]), gs);
        }
        out[0] = gs * delta;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) out[1 + ch] = w > 0.f ? g[ch] * w * c[ch] * (1.f - c[ch]) : 0.f;
        if constexpr (RS == 8) {
            out[4] = d[0];
            out[5] = d[1];
            out[6] = d[2];
            out[7] = 0.f;
        }
        if ((uint64_t)off0 + s0 < (uint64_t)n_rows) {
            float4* dst = reinterpret_cast<float4*>(rows + ((int64_t)off0 + s0) * RS);
#pragma unroll
            for (int q = 0; q < RS / 4; ++q) dst[q] = make_float4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
        }
        S = Sn;
        T = Tn;
        A0 = A1;
        B0 = B1;
        s0 = s1;
        ok0 = ok1;
        off0 = off1;
        A1 = A2;
        B1 = B2;
        s1 = s2;
    }
}

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t seg_records_bytes(int64_t n, int cap) {
    return 256 + 2 * up256((size_t)n * 4) + up256((size_t)cap * n * 16) + up256((size_t)cap * n * 8) +
           up256((size_t)cap * n * 4);
}

SegRecords seg_records_view(void* base, int64_t n, size_t bytes) {
    SegRecords r;
    if (n <= 0) return r;
    // the largest cap the buffer holds
    int cap = 0;
    for (int c = SEG_CAP_MAX; c >= 1; c = c > 8 ? c - 8 : c - 1)
        if (seg_records_bytes(n, c) <= bytes) {
            cap = c;
            break;
        }
    if (cap == 0) return r;
    char* p = static_cast<char*>(base);
    r.overflow = reinterpret_cast<uint32_t*>(p);
    r.total = r.overflow + 1;
    p += 256;
    r.count = reinterpret_cast<int32_t*>(p);
    p += up256((size_t)n * 4);
    r.olist = reinterpret_cast<int32_t*>(p);
    p += up256((size_t)n * 4);
    r.a = reinterpret_cast<float4*>(p);
    p += up256((size_t)cap * n * 16);
    r.b = reinterpret_cast<float2*>(p);
    p += up256((size_t)cap * n * 8);
    r.slot = reinterpret_cast<uint32_t*>(p);
    r.n = n;
    r.cap = cap;
    return r;
}

// Rows of leaf l's bucket: the recorded region (base0, or none), then the rows
// the second region's cursor handed out (never more than it holds).
__device__ __forceinline__ uint32_t bucket_rows(int64_t l, const uint32_t* __restrict__ base0,
                                                const uint32_t* __restrict__ count,
                                                const uint32_t* __restrict__ cursor) {
    return (base0 ? base0[l] : 0u) + min(count[l], cursor[l]);
}

// One bucket row added to a leaf's sums: dsigma and, per channel, a_ch Y_k(d_row).
template <int DEG>
__device__ __forceinline__ void bucket_add_row(const float4 h, const float4 q, float& gs, float* acc) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int RS = bwd_row_floats<DEG>();
    float Y[K];
    if constexpr (RS == 8)
        sh_basis<DEG>(q.x, q.y, q.z, Y);
    else
        sh_basis<DEG>(0.f, 0.f, 1.f, Y);
    gs += h.x;
    const float a[3] = {h.y, h.z, h.w};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[ch * K + k] += a[ch] * Y[k];
}

// Sum of the m rows at p taken by one thread (a light bucket), into gs/acc
// (zeroed by the caller).
template <int DEG>
__device__ __forceinline__ void bucket_sum_thread(const float4* __restrict__ p, uint32_t m, float& gs, float* acc) {
    constexpr int Q = bwd_row_floats<DEG>() / 4;     // float4 per row
    constexpr int U = 4;                              // rows whose loads are issued together
    uint32_t r = 0;
    for (; r + U <= m; r += U) {
        float4 h[U], q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            h[u] = p[(int64_t)(r + u) * Q];
            q[u] = Q == 2 ? p[(int64_t)(r + u) * Q + (Q - 1)] : h[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) bucket_add_row<DEG>(h[u], q[u], gs, acc);
    }
    for (; r < m; ++r) {
        const float4 h = p[(int64_t)r * Q];
        bucket_add_row<DEG>(h, Q == 2 ? p[(int64_t)r * Q + (Q - 1)] : h, gs, acc);
    }
}

// Sum of the m rows at p taken by a whole wave (called by all its lanes with
// the same p and m): lanes stride over the rows (consecutive lanes read
// consecutive rows), then a butterfly leaves the totals in every lane.
template <int DEG>
__device__ __forceinline__ void bucket_sum_wave(const float4* __restrict__ p, uint32_t m, float& gs, float* acc) {
    constexpr int NV = 3 * (DEG + 1) * (DEG + 1);
    constexpr int Q = bwd_row_floats<DEG>() / 4;
    constexpr int U = 4;          // rows per lane whose loads are issued together
    const int lane = threadIdx.x & (WAVE - 1);
    gs = 0.f;
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.f;
    uint32_t r = lane;
    for (; r + (U - 1) * WAVE < m; r += U * WAVE) {
        float4 h[U], q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            h[u] = p[(int64_t)(r + u * WAVE) * Q];
            q[u] = Q == 2 ? p[(int64_t)(r + u * WAVE) * Q + (Q - 1)] : h[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) bucket_add_row<DEG>(h[u], q[u], gs, acc);
    }
    for (; r < m; r += WAVE) {
        const float4 h = p[(int64_t)r * Q];
        bucket_add_row<DEG>(h, Q == 2 ? p[(int64_t)r * Q + (Q - 1)] : h, gs, acc);
    }
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        gs += __shfl_xor(gs, off, WAVE);
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += __shfl_xor(acc[j], off, WAVE);
    }
}

// Buckets of more rows than this are left out of the thread-per-leaf sums and
// reduced a wave per leaf by bwd_heavy_kernel: a thread-per-leaf sum would keep
// the block waiting on its longest bucket (a few leaves of a large batch
// collect thousands of rows).
constexpr uint32_t kLightRows = 64;

// Rows of the bucket of leaf l (0 for l >= L) and, for a light bucket, its sums
// (zero otherwise).
template <int DEG>
__device__ __forceinline__ uint32_t bucket_sum_light(int64_t l, int64_t L, const uint32_t* __restrict__ offset,
                                                     const uint32_t* __restrict__ base0,
                                                     const uint32_t* __restrict__ count,
                                                     const uint32_t* __restrict__ cursor,
                                                     const float* __restrict__ rows, float& gs, float* acc) {
    constexpr int NV = 3 * (DEG + 1) * (DEG + 1);
    constexpr int RS = bwd_row_floats<DEG>();
    const uint32_t m = l < L ? bucket_rows(l, base0, count, cursor) : 0u;
    gs = 0.f;
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.f;
    if (m > 0 && m <= kLightRows)
        bucket_sum_thread<DEG>(reinterpret_cast<const float4*>(rows + (int64_t)offset[l] * RS), m, gs, acc);
    return m;
}

// A fused optimiser step, by value: RMSProp (d1 = alpha) or Adam (d1, d2 =
// beta1, beta2; bc1, bc2 = its bias corrections; m_* = first moments).
enum { OPT_NONE = 0, OPT_RMSPROP = 1, OPT_ADAM = 2 };
struct FusedOpt {
    float lr_sigma, lr_sh, eps, d1, d2, bc1, bc2;
    float *m_sigma, *m_sh, *v_sigma, *v_sh;
};

template <int OPT>
__device__ __forceinline__ void opt_apply(float& th, float& m, float& v, float g, float lr, const FusedOpt& o) {
    if constexpr (OPT == OPT_ADAM)
        adam_update(th, m, v, g, lr, o.d1, o.d2, o.eps, o.bc1, o.bc2);
    else
        rmsprop_update(th, v, g, lr, o.d1, o.eps);
}

// theta[ti], v[si] (and Adam's m[si]) updated in place with gradient g
template <int OPT>
__device__ __forceinline__ void fused_update(float* theta, int64_t ti, float* m, float* v, int64_t si, float g,
                                             float lr, const FusedOpt& o) {
    float th = theta[ti], vv = v[si], mm = 0.f;
    if constexpr (OPT == OPT_ADAM) mm = m[si];
    opt_apply<OPT>(th, mm, vv, g, lr, o);
    if constexpr (OPT == OPT_ADAM) m[si] = mm;
    theta[ti] = th;
    v[si] = vv;
}

// A leaf's bucket totals (held by every lane of the wave) applied by the wave:
// lane k owns SH column k and lane 0 sigma.  A fused optimiser step updates
// the leaf; otherwise the sums are added to the gradient arrays when the
// bucket has rows.
template <int DEG, int OPT>
__device__ __forceinline__ void wave_leaf_apply(int64_t l, uint32_t m, float gs, const float* acc,
                                                float* __restrict__ gsig, float* __restrict__ gsh,
                                                float* __restrict__ sigma, float* __restrict__ sh, int stride,
                                                const FusedOpt& o) {
    constexpr int NV = 3 * (DEG + 1) * (DEG + 1);
    static_assert(NV <= WAVE, "one lane per column");
    const int lane = threadIdx.x & (WAVE - 1);
    float mine = 0.f;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (lane == j) mine = acc[j];
    if constexpr (OPT != OPT_NONE) {
        if (lane < NV) fused_update<OPT>(sh, l * stride + lane, o.m_sh, o.v_sh, l * NV + lane, mine, o.lr_sh, o);
        if (lane == 0) fused_update<OPT>(sigma, l, o.m_sigma, o.v_sigma, l, gs, o.lr_sigma, o);
    } else if (m > 0) {
        if (lane < NV && mine != 0.f) gsh[l * NV + lane] += mine;
        if (lane == 0) gsig[l] += gs;
    }
}

// The heavy buckets among the wave's leaves (lane i owns leaf l_i, whose
// bucket has m_i rows), one leaf at a time by all lanes.  Called by every
// lane of the wave.
template <int DEG, int OPT>
__device__ __forceinline__ void wave_heavy_leaves(int64_t l, uint32_t m, const uint32_t* __restrict__ offset,
                                                  const float* __restrict__ rows, float* __restrict__ gsig,
                                                  float* __restrict__ gsh, float* __restrict__ sigma,
                                                  float* __restrict__ sh, int stride, const FusedOpt& o) {
    constexpr int NV = 3 * (DEG + 1) * (DEG + 1);
    constexpr int RS = bwd_row_floats<DEG>();
    uint64_t heavy = __ballot(m > kLightRows);
    while (heavy) {
        const int j = __ffsll((unsigned long long)heavy) - 1;
        heavy &= heavy - 1;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)l, j);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)l >> 32), j);
        const int64_t lj = (int64_t)(((uint64_t)hi << 32) | lo);
        const uint32_t mj = (uint32_t)__builtin_amdgcn_readlane((int)m, j);
        float gs, acc[NV];
        bucket_sum_wave<DEG>(reinterpret_cast<const float4*>(rows + (int64_t)offset[lj] * RS), mj, gs, acc);
        wave_leaf_apply<DEG, OPT>(lj, mj, gs, acc, gsig, gsh, sigma, sh, stride, o);
    }
}

// Bucket reductions: one thread per leaf sums its bucket into registers, then
// the block stages the SH sums of its 256 leaves in LDS one channel at a time
// (K floats per leaf, padded to K + 1 against bank conflicts; 17 KB at degree
// 3, so several blocks stay resident per CU) and all threads walk that
// channel's columns of the block's leaves, so loads and stores are coalesced
// in K-float runs (a thread-per-leaf row of 3K floats would touch a new cache
// line per lane and instruction).  Heavy buckets are left out of that pass
// (their leaves are neither read nor written) for bwd_heavy_kernel.
constexpr int RED_BLOCK = 256;

template <int DEG>
__global__ __launch_bounds__(RED_BLOCK) void bwd_reduce_kernel(int64_t L, const uint32_t* __restrict__ offset,
                                                               const uint32_t* __restrict__ base0,
                                                               const uint32_t* __restrict__ count,
                                                               const uint32_t* __restrict__ cursor,
                                                               const float* __restrict__ rows,
                                                               float* __restrict__ gsig, float* __restrict__ gsh) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int NV = 3 * K;
    constexpr int KP = K + 1;
    __shared__ float stage[RED_BLOCK * KP];
    const int64_t l0 = (int64_t)blockIdx.x * RED_BLOCK;
    const int64_t l = l0 + threadIdx.x;
    float gs, acc[NV];
    const uint32_t m = bucket_sum_light<DEG>(l, L, offset, base0, count, cursor, rows, gs, acc);
    if (m > 0 && m <= kLightRows) gsig[l] += gs;
    const int64_t nl = L - l0 < RED_BLOCK ? L - l0 : RED_BLOCK;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        if (ch) __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) stage[threadIdx.x * KP + k] = acc[ch * K + k];
        __syncthreads();
        // a heavy leaf's staged sums are zero: none of its columns is written here
        for (int i = threadIdx.x; i < nl * K; i += RED_BLOCK) {
            const int r = i / K, k = i - r * K;
            const float v = stage[r * KP + k];
            if (v != 0.f) gsh[(l0 + r) * NV + ch * K + k] += v;
        }
    }
}

// The optimiser step on columns [ch K, ch K + K) of a block's nl leaves (rows
// of NV), whose SH sums sit in stage (K per leaf, padded to KP).  Item i =
// (leaf r, run q) covers W consecutive columns (W = 4: float4 accesses, when
// K % 4 == 0 and the planes are 16-byte aligned).  hit[r] = 0 marks a leaf with an empty bucket (g = 0):
// RMSProp then leaves its values exactly as they are (lr 0 / (sqrt(v) + eps)
// = 0) and only decays the square average, so the values are neither read
// nor written; Adam still moves such a leaf by its first moment.  hit[r] = 2
// marks a heavy bucket, whose leaf bwd_heavy_kernel updates.
template <int K, int NV, int W, int OPT>
__device__ __forceinline__ void fused_channel(int64_t l0, int nl, int ch, const float* stage, const int* hit,
                                              float* __restrict__ sh, int stride, const FusedOpt& o) {
    constexpr int KP = K + 1;
    constexpr int Q = K / W;
    static_assert(K % W == 0, "runs tile the channel");
    struct alignas(4 * W) Run {
        float x[W];
    };
    // two items per iteration, both items' loads issued before either update
    constexpr int U = 2;
    const int ni = nl * Q;
    for (int i0 = threadIdx.x; i0 < ni; i0 += U * RED_BLOCK) {
        Run v[U], th[U], m[U];
        bool live[U], full[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * RED_BLOCK;
            live[u] = i < ni && hit[i / Q] != 2;
            full[u] = false;
            if (live[u]) {
                const int r = i / Q, q = i - r * Q;
                const int64_t col = (int64_t)ch * K + q * W;
                v[u] = *reinterpret_cast<const Run*>(o.v_sh + (l0 + r) * NV + col);
                full[u] = !(OPT == OPT_RMSPROP && !hit[r]);
                if (full[u]) {
                    th[u] = *reinterpret_cast<const Run*>(sh + (l0 + r) * stride + col);
                    if constexpr (OPT == OPT_ADAM) m[u] = *reinterpret_cast<const Run*>(o.m_sh + (l0 + r) * NV + col);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!live[u]) continue;
            const int i = i0 + u * RED_BLOCK;
            const int r = i / Q, q = i - r * Q;
            const int64_t col = (int64_t)ch * K + q * W;
            if (!full[u]) {
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    float t0 = 0.f, m0 = 0.f;
                    opt_apply<OPT>(t0, m0, v[u].x[e], 0.f, o.lr_sh, o);
                }
            } else {
                Run mm{};
                if constexpr (OPT == OPT_ADAM) mm = m[u];
#pragma unroll
                for (int e = 0; e < W; ++e)
                    opt_apply<OPT>(th[u].x[e], mm.x[e], v[u].x[e], stage[r * KP + q * W + e], o.lr_sh, o);
                *reinterpret_cast<Run*>(sh + (l0 + r) * stride + col) = th[u];
                if constexpr (OPT == OPT_ADAM) *reinterpret_cast<Run*>(o.m_sh + (l0 + r) * NV + col) = mm;
            }
            *reinterpret_cast<Run*>(o.v_sh + (l0 + r) * NV + col) = v[u];
        }
    }
}

// The same reduction feeding the optimiser for every leaf (untouched leaves
// have g = 0: RMSProp only decays their square averages, Adam still moves
// them by its decayed first moment).
template <int DEG, int OPT, int W>
__global__ __launch_bounds__(RED_BLOCK) void bwd_fused_kernel(int64_t L, const uint32_t* __restrict__ offset,
                                                              const uint32_t* __restrict__ base0,
                                                              const uint32_t* __restrict__ count,
                                                              const uint32_t* __restrict__ cursor,
                                                              const float* __restrict__ rows,
                                                              float* __restrict__ sigma, float* __restrict__ sh,
                                                              int stride, FusedOpt o) {
    constexpr int NV = 3 * (DEG + 1) * (DEG + 1);
    // the sums of all 3K columns staged at once, so every row of the state is
    // swept in one pass (per channel, the half-lines a row shares with the
    // next channel were fetched again once the L2 had dropped them)
    constexpr int KC = NV, KP = KC + 1;
    __shared__ float stage[RED_BLOCK * KP];
    __shared__ int hit[RED_BLOCK];
    const int64_t l0 = (int64_t)blockIdx.x * RED_BLOCK;
    const int64_t l = l0 + threadIdx.x;
    float gs, acc[NV];
    const uint32_t m = bucket_sum_light<DEG>(l, L, offset, base0, count, cursor, rows, gs, acc);
    const bool heavy = m > kLightRows;
    if (l < L) {
        hit[threadIdx.x] = heavy ? 2 : (m > 0 ? 1 : 0);
        if (heavy) {
            // left to bwd_heavy_kernel
        } else if (OPT == OPT_RMSPROP && m == 0) {
            float th = 0.f, mm = 0.f;         // g = 0: sigma stays, its square average decays
            opt_apply<OPT>(th, mm, o.v_sigma[l], 0.f, o.lr_sigma, o);
        } else {
            fused_update<OPT>(sigma, l, o.m_sigma, o.v_sigma, l, gs, o.lr_sigma, o);
        }
    }
    const int64_t nl = L - l0 < RED_BLOCK ? L - l0 : RED_BLOCK;
#pragma unroll
    for (int k = 0; k < KC; ++k) stage[threadIdx.x * KP + k] = acc[k];
    __syncthreads();
    fused_channel<KC, NV, W, OPT>(l0, (int)nl, 0, stage, hit, sh, stride, o);
}

// Heavy buckets on average (many rows per leaf, e.g. a small tree under a
// large batch): one wave per leaf for every leaf.
template <int DEG, int OPT>
__global__ __launch_bounds__(RED_BLOCK) void bwd_reduce_wave_kernel(
    int64_t L, const uint32_t* __restrict__ offset, const uint32_t* __restrict__ base0,
    const uint32_t* __restrict__ count, const uint32_t* __restrict__ cursor, const float* __restrict__ rows,
    float* __restrict__ gsig, float* __restrict__ gsh, float* __restrict__ sigma, float* __restrict__ sh, int stride,
    FusedOpt o) {
    constexpr int NV = 3 * (DEG + 1) * (DEG + 1);
    constexpr int RS = bwd_row_floats<DEG>();
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    for (int64_t l = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; l < L; l += nw) {
        const uint32_t m = bucket_rows(l, base0, count, cursor);
        float gs, acc[NV];
        bucket_sum_wave<DEG>(reinterpret_cast<const float4*>(rows + (int64_t)offset[l] * RS), m, gs, acc);
        wave_leaf_apply<DEG, OPT>(l, m, gs, acc, gsig, gsh, sigma, sh, stride, o);
    }
}

// The heavy buckets the block reductions leave out: wave w of nw takes the
// leaves w + nw i, 64 at a time (lane j: i = b + j), so a run of adjacent
// heavy leaves (neighbours in space collect rows together) spreads over
// neighbouring waves instead of queueing in one.
template <int DEG, int OPT>
__global__ __launch_bounds__(RED_BLOCK) void bwd_heavy_kernel(
    int64_t L, const uint32_t* __restrict__ offset, const uint32_t* __restrict__ base0,
    const uint32_t* __restrict__ count, const uint32_t* __restrict__ cursor, const float* __restrict__ rows,
    float* __restrict__ gsig, float* __restrict__ gsh, float* __restrict__ sigma, float* __restrict__ sh, int stride,
    FusedOpt o) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    for (int64_t b = 0; w + nw * b < L; b += WAVE) {
        const int64_t l = w + nw * (b + lane);
        const uint32_t m = l < L ? bucket_rows(l, base0, count, cursor) : 0u;
        wave_heavy_leaves<DEG, OPT>(l, m, offset, rows, gsig, gsh, sigma, sh, stride, o);
    }
}

static FusedOpt fused_opt(const BwdArgs& a) {
    FusedOpt o{};
    o.m_sigma = a.m_sigma;
    o.m_sh = a.m_sh;
    o.v_sigma = a.v_sigma;
    o.v_sh = a.v_sh;
    if (a.adam) {
        o.lr_sigma = a.adam->lr_sigma;
        o.lr_sh = a.adam->lr_sh;
        o.eps = a.adam->eps;
        o.d1 = a.adam->beta1;
        o.d2 = a.adam->beta2;
        adam_bias_corrections(*a.adam, o.bc1, o.bc2);
    } else if (a.rms) {
        o.lr_sigma = a.rms->lr_sigma;
        o.lr_sh = a.rms->lr_sh;
        o.eps = a.rms->eps;
        o.d1 = a.rms->alpha;
    }
    return o;
}

static int opt_kind(const BwdArgs& a) { return a.adam ? OPT_ADAM : a.rms ? OPT_RMSPROP : OPT_NONE; }

// HEAVY: bwd_heavy_kernel (the buckets a block reduction left out), else
// bwd_reduce_wave_kernel (every leaf)
template <int DEG, int OPT, bool HEAVY>
static void launch_wave_opt(const dot_tree& t, const BwdArgs& a, const uint32_t* offset, const uint32_t* base0,
                            const uint32_t* count, const uint32_t* cursor, const float* rows, hipStream_t s) {
    const int64_t L = t.n_leaves;
    const int64_t want = HEAVY ? (L + RED_BLOCK - 1) / RED_BLOCK : (L + RED_BLOCK / WAVE - 1) / (RED_BLOCK / WAVE);
    const unsigned g = (unsigned)std::min<int64_t>(want, HEAVY ? 2048 : 1 << 16);
    float* gsig = OPT == OPT_NONE ? a.grad_sigma : nullptr;
    float* gsh = OPT == OPT_NONE ? a.grad_sh : nullptr;
    float* sg = OPT == OPT_NONE ? nullptr : static_cast<float*>(t.sigma);
    float* sh = OPT == OPT_NONE ? nullptr : static_cast<float*>(t.sh);
    const FusedOpt o = OPT == OPT_NONE ? FusedOpt{} : fused_opt(a);
    if constexpr (HEAVY)
        hipLaunchKernelGGL((bwd_heavy_kernel<DEG, OPT>), dim3(g), dim3(RED_BLOCK), 0, s, L, offset, base0, count,
                           cursor, rows, gsig, gsh, sg, sh, t.sh_stride, o);
    else
        hipLaunchKernelGGL((bwd_reduce_wave_kernel<DEG, OPT>), dim3(g), dim3(RED_BLOCK), 0, s, L, offset, base0,
                           count, cursor, rows, gsig, gsh, sg, sh, t.sh_stride, o);
}

template <int DEG, bool HEAVY>
static void launch_wave(const dot_tree& t, const BwdArgs& a, const uint32_t* offset, const uint32_t* base0,
                        const uint32_t* count, const uint32_t* cursor, const float* rows, hipStream_t s) {
    switch (opt_kind(a)) {
        case OPT_RMSPROP: launch_wave_opt<DEG, OPT_RMSPROP, HEAVY>(t, a, offset, base0, count, cursor, rows, s); break;
        case OPT_ADAM: launch_wave_opt<DEG, OPT_ADAM, HEAVY>(t, a, offset, base0, count, cursor, rows, s); break;
        default: launch_wave_opt<DEG, OPT_NONE, HEAVY>(t, a, offset, base0, count, cursor, rows, s); break;
    }
}

// buckets holding at least this many rows on average are reduced a wave per leaf
static constexpr uint32_t kWaveRowsPerLeaf = 32;

// p[0, n) = 0, and *word = 0 when given (one launch for an array and a counter)
__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t* word, int n_words) {
    if (word && blockIdx.x == 0 && (int)threadIdx.x < n_words) word[threadIdx.x] = 0u;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s, uint32_t* word, int n_words) {
    if (n <= 0 && !word) return hipSuccess;
    const int64_t g = std::max<int64_t>((n + 255) / 256, 1);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<int64_t>(g, 65536)), dim3(256), 0, s, p, n, word,
                       n_words < 1 ? 1 : (n_words > 256 ? 256 : n_words));
    return hipGetLastError();
}

template <int DT, int DEG>
static hipError_t fwd_dispatch_stats(const TreeView& tv, const RayBatch& rb, const FwdArgs& a,
                                     dim3 grid, hipStream_t s) {
    if (a.stats)
        hipLaunchKernelGGL((render_fwd_kernel<DT, DEG, 1>), grid, dim3(BLOCK), 0, s, tv, rb, a);
    else if constexpr (DT == DOT_F32) {
        if (a.leaf_count)
            hipLaunchKernelGGL((render_fwd_kernel<DT, DEG, 2>), grid, dim3(BLOCK), 0, s, tv, rb, a);
        else
            hipLaunchKernelGGL((render_fwd_kernel<DT, DEG, 0>), grid, dim3(BLOCK), 0, s, tv, rb, a);
    } else {
        hipLaunchKernelGGL((render_fwd_kernel<DT, DEG, 0>), grid, dim3(BLOCK), 0, s, tv, rb, a);
    }
    return hipGetLastError();
}

template <int DT>
static hipError_t fwd_dispatch_deg(int deg, const TreeView& tv, const RayBatch& rb, const FwdArgs& a,
                                   dim3 grid, hipStream_t s) {
    switch (deg) {
        case 0: return fwd_dispatch_stats<DT, 0>(tv, rb, a, grid, s);
        case 1: return fwd_dispatch_stats<DT, 1>(tv, rb, a, grid, s);
        case 2: return fwd_dispatch_stats<DT, 2>(tv, rb, a, grid, s);
        default: return fwd_dispatch_stats<DT, 3>(tv, rb, a, grid, s);
    }
}

hipError_t launch_render_fwd(const dot_tree& t, const RayBatch& rb, const FwdArgs& a, hipStream_t s) {
    if (rb.n_tiles == 0) return hipSuccess;
    dim3 grid((unsigned)((rb.n_tiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
    TreeView tv = t.view();
    switch (t.storage) {
        case DOT_F32: return fwd_dispatch_deg<DOT_F32>(t.degree, tv, rb, a, grid, s);
        case DOT_F16: return fwd_dispatch_deg<DOT_F16>(t.degree, tv, rb, a, grid, s);
        case DOT_PAL16: return fwd_dispatch_deg<DOT_PAL16>(t.degree, tv, rb, a, grid, s);
        default: return fwd_dispatch_deg<DOT_BF16>(t.degree, tv, rb, a, grid, s);
    }
}

template <int DT>
static hipError_t bwd_dispatch_deg(int deg, const TreeView& tv, const RayBatch& rb, const BwdArgs& a,
                                   dim3 grid, hipStream_t s) {
    switch (deg) {
        case 0: hipLaunchKernelGGL((render_bwd_kernel<DT, 0>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
        case 1: hipLaunchKernelGGL((render_bwd_kernel<DT, 1>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
        case 2: hipLaunchKernelGGL((render_bwd_kernel<DT, 2>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
        default: hipLaunchKernelGGL((render_bwd_kernel<DT, 3>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
    }
    return hipGetLastError();
}

template <int DT>
static hipError_t bwd_wave_dispatch_deg(int deg, const TreeView& tv, const RayBatch& rb, const BwdArgs& a,
                                        dim3 grid, hipStream_t s) {
    switch (deg) {
        case 0: hipLaunchKernelGGL((render_bwd_wave_kernel<DT, 0>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
        case 1: hipLaunchKernelGGL((render_bwd_wave_kernel<DT, 1>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
        case 2: hipLaunchKernelGGL((render_bwd_wave_kernel<DT, 2>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
        default: hipLaunchKernelGGL((render_bwd_wave_kernel<DT, 3>), grid, dim3(BLOCK), 0, s, tv, rb, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_render_bwd_wave(const dot_tree& t, const RayBatch& rb, const BwdArgs& a, hipStream_t s) {
    if (rb.n_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)((rb.n_tiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
    TreeView tv = t.view();
    switch (t.storage) {
        case DOT_F32: return bwd_wave_dispatch_deg<DOT_F32>(t.degree, tv, rb, a, grid, s);
        case DOT_F16: return bwd_wave_dispatch_deg<DOT_F16>(t.degree, tv, rb, a, grid, s);
        default: return bwd_wave_dispatch_deg<DOT_BF16>(t.degree, tv, rb, a, grid, s);
    }
}

static hipError_t bwd_atomic(const dot_tree& t, const RayBatch& rb, const BwdArgs& a, dim3 grid, hipStream_t s) {
    TreeView tv = t.view();
    switch (t.storage) {
        case DOT_F32: return bwd_dispatch_deg<DOT_F32>(t.degree, tv, rb, a, grid, s);
        case DOT_F16: return bwd_dispatch_deg<DOT_F16>(t.degree, tv, rb, a, grid, s);
        default: return bwd_dispatch_deg<DOT_BF16>(t.degree, tv, rb, a, grid, s);
    }
}

template <int DT>
static void launch_emit(int deg, const TreeView& tv, const RayBatch& rb, const BwdArgs& a, const uint32_t* off,
                        const uint32_t* b0, const uint32_t* cnt, uint32_t* cur, float* rows, dim3 grid, hipStream_t s) {
    switch (deg) {
        case 0: hipLaunchKernelGGL((bwd_emit_kernel<DT, 0>), grid, dim3(BLOCK), 0, s, tv, rb, a, off, b0, cnt, cur, rows); break;
        case 1: hipLaunchKernelGGL((bwd_emit_kernel<DT, 1>), grid, dim3(BLOCK), 0, s, tv, rb, a, off, b0, cnt, cur, rows); break;
        case 2: hipLaunchKernelGGL((bwd_emit_kernel<DT, 2>), grid, dim3(BLOCK), 0, s, tv, rb, a, off, b0, cnt, cur, rows); break;
        default: hipLaunchKernelGGL((bwd_emit_kernel<DT, 3>), grid, dim3(BLOCK), 0, s, tv, rb, a, off, b0, cnt, cur, rows); break;
    }
}

// c = a + b elementwise (a bucket's two regions) and z = 0 (the bucket
// cursors); the first thread also copies *w_src to *w_dst (a word the host
// reads back together with the scan total)
__global__ void add_u32_kernel(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, uint32_t* __restrict__ c,
                               uint32_t* __restrict__ z, int64_t n, const uint32_t* __restrict__ w_src,
                               uint32_t* __restrict__ w_dst) {
    if (w_src && blockIdx.x == 0 && threadIdx.x == 0) *w_dst = *w_src;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        c[i] = a[i] + b[i];
        z[i] = 0u;
    }
}

// bucket scratch beyond this many bytes falls back to the atomic adjoint
static constexpr double kBucketBytesMax = 8.0 * (1ull << 30);

static hipError_t bwd_fused_dense(const dot_tree& t, const RayBatch& rb, const BwdArgs& a0, dim3 grid, hipStream_t s);
static hipError_t launch_fused_zero_grad(const dot_tree& t, const BwdArgs& a, hipStream_t s) {
    RayBatch none{};
    return bwd_fused_dense(t, none, a, dim3(1), s);
}

// Fused path when the buckets cannot be used: dense gradients from the atomic
// adjoint, then the elementwise optimiser step.
static hipError_t bwd_fused_dense(const dot_tree& t, const RayBatch& rb, const BwdArgs& a0, dim3 grid, hipStream_t s) {
    const int nv = 3 * (t.degree + 1) * (t.degree + 1);
    float* g = static_cast<float*>(t.alloc.get((size_t)t.n_leaves * (1 + nv) * 4));
    if (!g) return hipErrorOutOfMemory;
    BwdArgs a = a0;
    a.grad_sigma = g;
    a.grad_sh = g + t.n_leaves;
    const int64_t n = t.n_leaves * (1 + nv);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(g), n, nullptr, 1);
    hipError_t e = rb.n_tiles ? bwd_atomic(t, rb, a, grid, s) : hipGetLastError();
    if (e == hipSuccess)
        e = a.adam ? launch_adam(t, a.grad_sigma, a.grad_sh, a.m_sigma, a.v_sigma, a.m_sh, a.v_sh, *a.adam, s)
                   : launch_rmsprop(t, a.grad_sigma, a.grad_sh, a.v_sigma, a.v_sh, *a.rms, s);
    t.alloc.put(g);
    return e;
}

template <int DEG>
static void launch_bwd_fused(const dot_tree& t, const BwdArgs& a, const uint32_t* offset, const uint32_t* base0,
                             const uint32_t* count, const uint32_t* cursor, const float* rows, hipStream_t s) {
    const int64_t L = t.n_leaves;
    const unsigned rg = (unsigned)((L + RED_BLOCK - 1) / RED_BLOCK);
    constexpr int K = (DEG + 1) * (DEG + 1);
    float* sg = static_cast<float*>(t.sigma);
    float* sh = static_cast<float*>(t.sh);
    const FusedOpt o = fused_opt(a);
    auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const bool vec = K % 4 == 0 && t.sh_stride % 4 == 0 && a16(sh) && a16(o.v_sh) && (!a.adam || a16(o.m_sh));
    const dim3 g(rg), b(RED_BLOCK);
    if constexpr (K % 4 == 0) {
        if (vec) {
            if (a.adam)
                hipLaunchKernelGGL((bwd_fused_kernel<DEG, OPT_ADAM, 4>), g, b, 0, s, L, offset, base0, count, cursor,
                                   rows, sg, sh, t.sh_stride, o);
            else
                hipLaunchKernelGGL((bwd_fused_kernel<DEG, OPT_RMSPROP, 4>), g, b, 0, s, L, offset, base0, count,
                                   cursor, rows, sg, sh, t.sh_stride, o);
            return;
        }
    }
    if (a.adam)
        hipLaunchKernelGGL((bwd_fused_kernel<DEG, OPT_ADAM, 1>), g, b, 0, s, L, offset, base0, count, cursor, rows, sg,
                           sh, t.sh_stride, o);
    else
        hipLaunchKernelGGL((bwd_fused_kernel<DEG, OPT_RMSPROP, 1>), g, b, 0, s, L, offset, base0, count, cursor, rows,
                           sg, sh, t.sh_stride, o);
}

void note_forward(const dot_tree& t, const SegRecords& rec, const uint32_t* counts, int64_t n_rays, hipStream_t s) {
    if (!t.note_words) {
        void* h = nullptr;
        if (hipHostMalloc(&h, sizeof(uint32_t) * 2 * dot_tree::kNotes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        t.note_words = static_cast<uint32_t*>(h);
    }
    const int i = t.note_next;
    t.note_next = (i + 1) % dot_tree::kNotes;
    dot_tree::FwdNote& nt = t.notes[i];
    // the slot's previous copy must have landed before it is written again
    if (nt.rec && nt.ev && hipEventSynchronize(nt.ev) != hipSuccess) (void)hipGetLastError();
    nt.rec = nullptr;
    if (!nt.ev && hipEventCreateWithFlags(&nt.ev, hipEventDisableTiming) != hipSuccess) {
        nt.ev = nullptr;
        (void)hipGetLastError();
        return;
    }
    if (hipMemcpyAsync(t.note_words + 2 * i, rec.overflow, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(nt.ev, s) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    nt.rec = rec.overflow;
    nt.counts = counts;
    nt.n_rays = n_rays;
    nt.n_leaves = t.n_leaves;
}

const uint32_t* find_note(const dot_tree& t, const void* rec, const uint32_t* counts, int64_t n_rays, hipEvent_t* ev) {
    if (!t.note_words) return nullptr;
    // the most recent forward into these buffers
    for (int k = 1; k <= dot_tree::kNotes; ++k) {
        const int i = (t.note_next - k + dot_tree::kNotes) % dot_tree::kNotes;
        const dot_tree::FwdNote& nt = t.notes[i];
        if (nt.rec == rec && nt.counts == counts && nt.n_rays == n_rays && nt.n_leaves == t.n_leaves && nt.ev) {
            *ev = nt.ev;
            return t.note_words + 2 * i;
        }
    }
    return nullptr;
}

void drop_notes(const dot_tree& t) {
    for (auto& nt : t.notes) {
        if (nt.ev) {
            (void)hipEventSynchronize(nt.ev);
            (void)hipEventDestroy(nt.ev);
        }
        nt = dot_tree::FwdNote{};
    }
    if (t.note_words) (void)hipHostFree(t.note_words);
    t.note_words = nullptr;
    t.note_next = 0;
}

hipError_t launch_render_bwd(const dot_tree& t, const RayBatch& rb, const BwdArgs& a, hipStream_t s) {
    const bool fused = opt_kind(a) != OPT_NONE;
    if (rb.n_tiles == 0) {
        // no rays: a fused step still runs with g = 0 (decaying moments)
        return fused ? launch_fused_zero_grad(t, a, s) : hipSuccess;
    }
    dim3 grid((unsigned)((rb.n_tiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
    const int64_t L = t.n_leaves;
    const int rs = bwd_row_floats_rt(t.degree);
    TreeView tv = t.view();
    // Bucket regions: with the training forward's counts and its records,
    // base0 = its recorded counts (rows the replay writes) and count = its
    // other counts; with its counts but no records, every segment goes through
    // the cursors, so there is no recorded region and count = the sum of the
    // two (a forward that recorded would otherwise leave its recorded region
    // unwritten); without counts, count = our own counting pass.  `total` =
    // all rows of a leaf's bucket, which feeds the scan.
    const bool replay = a.leaf_count && a.rec.a;
    const uint32_t* base0 = replay ? a.leaf_count : nullptr;
    uint32_t* count_own = a.leaf_count ? nullptr : static_cast<uint32_t*>(t.scratch_get((size_t)L * 4, s));
    uint32_t* total = a.leaf_count ? static_cast<uint32_t*>(t.scratch_get((size_t)L * 4, s)) : count_own;
    const uint32_t* count = replay ? a.leaf_count + L : total;
    uint32_t* offset = static_cast<uint32_t*>(t.scratch_get((size_t)L * 4, s));
    uint32_t* cursor = static_cast<uint32_t*>(t.scratch_get((size_t)L * 4, s));
    uint32_t* bsum = static_cast<uint32_t*>(t.scratch_get((size_t)scan_scratch_elems(L) * 4, s));
    uint32_t* tot = static_cast<uint32_t*>(t.scratch_get(16, s));
    auto drop = [&]() {
        t.scratch_put(count_own, s);
        if (a.leaf_count) t.scratch_put(total, s);
        t.scratch_put(offset, s);
        t.scratch_put(cursor, s);
        t.scratch_put(bsum, s);
        t.scratch_put(tot, s);
    };
    // Bucket offsets and the row total are 32-bit: a batch whose contributing
    // segments (at most max_steps per ray) could reach 2^32 takes the atomic
    // path instead, so a wrapped total can never size the rows.
    const bool fits32 = (double)rb.n_rays * (double)tv.max_steps < 4294967295.0;
    if (!fits32 || !total || !offset || !cursor || !bsum || !tot) {
        drop();
        return fused ? bwd_fused_dense(t, rb, a, grid, s) : bwd_atomic(t, rb, a, grid, s);
    }
    unsigned fg = (unsigned)std::min<int64_t>((L + 255) / 256, 65536);
    if (!a.leaf_count) {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(fg), dim3(256), 0, s, cursor, L, nullptr, 1);
        hipLaunchKernelGGL(fill_u32_kernel, dim3(fg), dim3(256), 0, s, count_own, L, nullptr, 1);
        switch (t.storage) {
            case DOT_F32: hipLaunchKernelGGL(bwd_count_kernel<DOT_F32>, grid, dim3(BLOCK), 0, s, tv, rb, a, count_own); break;
            case DOT_F16: hipLaunchKernelGGL(bwd_count_kernel<DOT_F16>, grid, dim3(BLOCK), 0, s, tv, rb, a, count_own); break;
            default: hipLaunchKernelGGL(bwd_count_kernel<DOT_BF16>, grid, dim3(BLOCK), 0, s, tv, rb, a, count_own); break;
        }
    }
    hipError_t e = hipSuccess;
    // tot[1] = the forward's overflow count (zero without records); small trees
    // sum the two count regions, clear the cursors and scan in one launch
    if (!a.leaf_count ||
        !scan_u32_sum2(a.leaf_count, a.leaf_count + L, total, cursor, offset, L, tot, a.rec.a ? a.rec.overflow : nullptr,
                       tot + 1, s, &e)) {
        if (a.leaf_count)
            hipLaunchKernelGGL(add_u32_kernel, dim3(fg), dim3(256), 0, s, a.leaf_count, a.leaf_count + L, total, cursor,
                               L, a.rec.a ? a.rec.overflow : nullptr, tot + 1);
        e = scan_u32(total, offset, L, bsum, tot, s);
    }
    // The row total and the overflow count: from the note of the forward that
    // recorded (its copy, queued behind that forward, is waited for by its event:
    // the stream keeps running), else in one copy into pinned memory and one wait.
    hipEvent_t note_ev = nullptr;
    const uint32_t* note = replay ? find_note(t, a.rec.overflow, a.leaf_count, rb.n_rays, &note_ev) : nullptr;
    uint32_t m = 0, overflow = 0;
    if (note) {
        if (e == hipSuccess) e = hipEventSynchronize(note_ev);
        overflow = note[0];
        m = note[1];
    } else {
        if (e == hipSuccess && !t.host_rb) {
            void* h = nullptr;
            e = hipHostMalloc(&h, 16, hipHostMallocDefault);
            if (e == hipSuccess) t.host_rb = static_cast<uint32_t*>(h);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(t.host_rb, tot, a.rec.a ? 8 : 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) {
            m = t.host_rb[0];
            overflow = a.rec.a ? t.host_rb[1] : 0u;
        }
    }
    if (e != hipSuccess) {
        drop();
        return e;
    }
    float* rows = nullptr;
    if ((double)m * rs * 4 <= kBucketBytesMax) rows = static_cast<float*>(t.scratch_get((size_t)std::max<uint32_t>(m, 1) * rs * 4, s));
    if (!rows) {
        drop();
        return fused ? bwd_fused_dense(t, rb, a, grid, s) : bwd_atomic(t, rb, a, grid, s);
    }
    BwdArgs ae = a;
    ae.n_rows = m;
    if (a.rec.a) {
        // replay the recorded segments; re-traverse only the rays with more
        switch (t.degree) {
            case 0: hipLaunchKernelGGL(bwd_emit_rec_kernel<0>, grid, dim3(BLOCK), 0, s, rb, a, L, offset, m, rows); break;
            case 1: hipLaunchKernelGGL(bwd_emit_rec_kernel<1>, grid, dim3(BLOCK), 0, s, rb, a, L, offset, m, rows); break;
            case 2: hipLaunchKernelGGL(bwd_emit_rec_kernel<2>, grid, dim3(BLOCK), 0, s, rb, a, L, offset, m, rows); break;
            default: hipLaunchKernelGGL(bwd_emit_rec_kernel<3>, grid, dim3(BLOCK), 0, s, rb, a, L, offset, m, rows); break;
        }
        if (overflow > 0) {
            // only FP32 trees record (training storage)
            const int64_t no = std::min<int64_t>(overflow, rb.n_rays);
            const dim3 lg((unsigned)((no + BLOCK - 1) / BLOCK));
            switch (t.degree) {
                case 0: hipLaunchKernelGGL((bwd_emit_list_kernel<DOT_F32, 0>), lg, dim3(BLOCK), 0, s, tv, rb, ae, a.rec.olist, no, offset, base0, count, cursor, rows); break;
                case 1: hipLaunchKernelGGL((bwd_emit_list_kernel<DOT_F32, 1>), lg, dim3(BLOCK), 0, s, tv, rb, ae, a.rec.olist, no, offset, base0, count, cursor, rows); break;
                case 2: hipLaunchKernelGGL((bwd_emit_list_kernel<DOT_F32, 2>), lg, dim3(BLOCK), 0, s, tv, rb, ae, a.rec.olist, no, offset, base0, count, cursor, rows); break;
                default: hipLaunchKernelGGL((bwd_emit_list_kernel<DOT_F32, 3>), lg, dim3(BLOCK), 0, s, tv, rb, ae, a.rec.olist, no, offset, base0, count, cursor, rows); break;
            }
        }
    } else {
        switch (t.storage) {
            case DOT_F32: launch_emit<DOT_F32>(t.degree, tv, rb, ae, offset, base0, count, cursor, rows, grid, s); break;
            case DOT_F16: launch_emit<DOT_F16>(t.degree, tv, rb, ae, offset, base0, count, cursor, rows, grid, s); break;
            default: launch_emit<DOT_BF16>(t.degree, tv, rb, ae, offset, base0, count, cursor, rows, grid, s); break;
        }
    }
    const unsigned rg = (unsigned)((L + RED_BLOCK - 1) / RED_BLOCK);
    const bool wave_all = (uint64_t)m >= (uint64_t)kWaveRowsPerLeaf * (uint64_t)L;
    if (wave_all) {
        switch (t.degree) {
            case 0: launch_wave<0, false>(t, a, offset, base0, count, cursor, rows, s); break;
            case 1: launch_wave<1, false>(t, a, offset, base0, count, cursor, rows, s); break;
            case 2: launch_wave<2, false>(t, a, offset, base0, count, cursor, rows, s); break;
            default: launch_wave<3, false>(t, a, offset, base0, count, cursor, rows, s); break;
        }
    } else if (fused) {
        switch (t.degree) {
            case 0: launch_bwd_fused<0>(t, a, offset, base0, count, cursor, rows, s); break;
            case 1: launch_bwd_fused<1>(t, a, offset, base0, count, cursor, rows, s); break;
            case 2: launch_bwd_fused<2>(t, a, offset, base0, count, cursor, rows, s); break;
            default: launch_bwd_fused<3>(t, a, offset, base0, count, cursor, rows, s); break;
        }
    } else switch (t.degree) {
        case 0: hipLaunchKernelGGL(bwd_reduce_kernel<0>, dim3(rg), dim3(RED_BLOCK), 0, s, L, offset, base0, count, cursor, rows, a.grad_sigma, a.grad_sh); break;
        case 1: hipLaunchKernelGGL(bwd_reduce_kernel<1>, dim3(rg), dim3(RED_BLOCK), 0, s, L, offset, base0, count, cursor, rows, a.grad_sigma, a.grad_sh); break;
        case 2: hipLaunchKernelGGL(bwd_reduce_kernel<2>, dim3(rg), dim3(RED_BLOCK), 0, s, L, offset, base0, count, cursor, rows, a.grad_sigma, a.grad_sh); break;
        default: hipLaunchKernelGGL(bwd_reduce_kernel<3>, dim3(rg), dim3(RED_BLOCK), 0, s, L, offset, base0, count, cursor, rows, a.grad_sigma, a.grad_sh); break;
    }
    // the heavy buckets a block reduction left out
    if (!wave_all) switch (t.degree) {
        case 0: launch_wave<0, true>(t, a, offset, base0, count, cursor, rows, s); break;
        case 1: launch_wave<1, true>(t, a, offset, base0, count, cursor, rows, s); break;
        case 2: launch_wave<2, true>(t, a, offset, base0, count, cursor, rows, s); break;
        default: launch_wave<3, true>(t, a, offset, base0, count, cursor, rows, s); break;
    }
    e = hipGetLastError();
    t.scratch_put(rows, s);
    drop();
    return e;
}

}  // namespace dot
