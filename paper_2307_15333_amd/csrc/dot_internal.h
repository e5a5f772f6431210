// Internal declarations of libdot (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include <cmath>
#include <cstdint>
#include <string>

#include "dot.h"

namespace dot {

// Lattice used by the traversal: 2^LAT cells per axis at the finest level,
// so a tree may be up to LAT levels deep (DOT_MAX_DEPTH).
constexpr int LAT = 16;
constexpr int LAT_N = 1 << LAT;
static_assert(LAT == DOT_MAX_DEPTH, "lattice depth must match the ABI depth limit");

// Elements per leaf row of the SH plane: 3K values padded to 16 bytes.
inline int sh_stride_for(int degree, int storage) {
    int nv = 3 * (degree + 1) * (degree + 1);
    int per16 = storage == DOT_F32 ? 4 : 8;
    return (nv + per16 - 1) / per16 * per16;
}
inline int storage_bytes(int storage) { return storage == DOT_F32 ? 4 : 2; }

// Face-neighbour links of the leaves.  links[6 * leaf + 2 * axis + (dir > 0)]
// names what lies across that face of the leaf, at the leaf's depth or above:
//   LINK_OUT                 the face is on the root cube's boundary;
//   bit 31 clear             an internal node of the same depth as the leaf;
//   bit 31 set               a leaf: bits 0-26 its id, bits 27-30 how many
//                            levels shallower than this leaf it is (0..15).
// A leaf's depth is at least 1 when the tree has internal nodes, so the depth
// difference fits in 4 bits; leaf ids need n_leaves < 2^27 - 1.
constexpr uint32_t LINK_OUT = 0xffffffffu;
constexpr uint32_t LINK_LEAF = 0x80000000u;
constexpr int LINK_ID_BITS = 27;
constexpr uint32_t LINK_ID_MASK = (1u << LINK_ID_BITS) - 1u;
constexpr int64_t LINK_MAX_LEAVES = (int64_t)LINK_ID_MASK;

// Everything a kernel needs to read a tree (passed by value).
struct TreeView {
    const int32_t* child;
    const void* sigma;
    const void* sh;
    int64_t n_internal;
    int64_t n_leaves;
    float bmin[3];
    float scale;      // lattice cells per world unit = LAT_N / bbox_size
    int max_steps;    // safety bound on traversal steps per ray
    int sh_stride;    // elements per SH row (of the palette for DOT_PAL16)
    const void* palette;   // DOT_PAL16: FP16 palette rows; `sh` holds uint16 indices
    const uint32_t* links; // face-neighbour links [n_leaves][6], or null (ancestor-stack walk)
};

struct Alloc {
    dot_allocator a{};
    bool custom = false;
    void* get(size_t bytes) const;
    void put(void* p) const;
};

}  // namespace dot

struct dot_tree {
    dot::Alloc alloc;
    int64_t n_internal = 0, n_leaves = 0;
    int32_t degree = 0, storage = 0, max_depth = 0, sh_stride = 0;
    float bmin[3] = {0, 0, 0};
    float size = 1.f;
    int32_t* child = nullptr;     // device
    void* sigma = nullptr;        // device
    void* sh = nullptr;           // device
    uint8_t* leaf_depth = nullptr;  // device
    void* palette = nullptr;        // device, DOT_PAL16 only
    int32_t palette_bits = 0;
    uint32_t* links = nullptr;      // device [n_leaves][6], null when off or not built
    bool links_on = true;           // keep face-neighbour links (rebuilt after refinement)
    // pinned host words the adjoint reads back (allocated on first use; one
    // adjoint at a time per tree, like every other call that uses its scratch)
    mutable uint32_t* host_rb = nullptr;
    // What each recent training forward that recorded hands its adjoint: the
    // batch's bucket-row total and overflow count, copied into pinned memory
    // behind an event by the forward, so the adjoint reads them without
    // stopping the stream.  Keyed by the records and counts buffers.
    struct FwdNote {
        const void* rec = nullptr;
        const uint32_t* counts = nullptr;
        int64_t n_rays = 0, n_leaves = 0;   // n_leaves: a refinement in between invalidates the note
        hipEvent_t ev = nullptr;
    };
    static constexpr int kNotes = 4;
    mutable FwdNote notes[kNotes];
    mutable uint32_t* note_words = nullptr;   // pinned [kNotes][2]: overflow, total
    mutable int note_next = 0;
    // Scratch of the per-step calls (the adjoint's buckets and scans), kept
    // for the next call on the same stream instead of going back to the
    // allocator after every call (with a caller's allocator that is a call
    // into the caller per block).  A block is reused only on the stream it was
    // last used on, so stream order protects it; at most kScratchKept are kept.
    struct ScratchBlock {
        void* p;
        size_t cap;
        hipStream_t s;
    };
    static constexpr size_t kScratchKept = 12;
    mutable std::vector<ScratchBlock> scratch_free, scratch_live;
    void* scratch_get(size_t bytes, hipStream_t s) const;
    void scratch_put(void* p, hipStream_t s) const;
    void scratch_clear() const;

    dot::TreeView view() const {
        dot::TreeView v;
        v.child = child;
        v.sigma = sigma;
        v.sh = sh;
        v.n_internal = n_internal;
        v.n_leaves = n_leaves;
        for (int a = 0; a < 3; ++a) v.bmin[a] = bmin[a];
        v.scale = (float)dot::LAT_N / size;
        int md = max_depth < 1 ? 1 : max_depth;
        v.max_steps = 3 * (1 << md) + 64;
        v.sh_stride = sh_stride;
        v.palette = palette;
        v.links = links;
        return v;
    }
};

namespace dot {

// thread-local error message
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define DOT_HIP(call)                                    \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return ::dot::hip_fail(e_, #call); \
    } while (0)

// ---- launchers (defined next to their kernels) ----

struct RayBatch {
    int kind;
    int n_cams;
    const dot_camera* cams;
    int width, height;
    int64_t n_rays;
    const int32_t* cam_idx;
    const int32_t* pix_idx;
    const float* origins;
    const float* dirs;
    int64_t n_tiles;   // 64-ray units
};

// Segment records of a training forward, replayed by the adjoint instead of a
// second traversal: per ray up to `cap` composited segments (sigma > 0), slot
// major ([slot][ray]) so one step's writes and reads are coalesced, each with
// the bucket slot the forward reserved for its gradient row.  A ray with more
// segments is listed; the adjoint replays its first `cap` and re-traverses it
// for the rest.  The buffer's size sets `cap`.
//
// Per-leaf counts of a training forward (uint32 [2][L]): [0][l] the recorded
// segments of leaf l (their rows take bucket slots 0 .. [0][l] - 1, reserved
// by the forward), [1][l] the other segments with sigma > 0 (slots after
// those, taken in the adjoint).  Bucket l holds [0][l] + [1][l] rows.
constexpr int SEG_CAP_MAX = 1024;
struct SegRecords {
    float4* a = nullptr;          // [cap][n]: leaf id bits, delta, tau, c0
    float2* b = nullptr;          // [cap][n]: c1, c2
    uint32_t* slot = nullptr;     // [cap][n]: bucket slot of the record's row
    int32_t* count = nullptr;     // [n]: records of the ray
    uint32_t* overflow = nullptr; // [1]: rays with more than `cap` records
    uint32_t* total = nullptr;    // [1]: segments with sigma > 0 of the batch (= bucket rows of its adjoint)
    int32_t* olist = nullptr;     // [n]: ids of those rays (first `overflow` entries)
    int64_t n = 0;                // rays the buffer holds (the slot stride)
    int cap = 0;                  // records per ray
};
size_t seg_records_bytes(int64_t n_rays, int cap);
// view of a buffer of `bytes` for n rays; cap = 0 when it is too small for one record
SegRecords seg_records_view(void* base, int64_t n_rays, size_t bytes);

struct FwdArgs {
    float* rgb;         // may be null
    int32_t* nseg;      // may be null
    float* signal;      // may be null
    int signal_mode;
    float bg[3];
    float thr;          // -ln(t_stop), +inf when disabled
    unsigned long long* stats;  // may be null
    uint32_t* leaf_count;       // may be null: [2][L] per-leaf segment counts (recorded, other) for the adjoint
    uint32_t* leaf_rest;        // leaf_count + L
    SegRecords rec;             // training forward: segment records (a == null: none)
};

struct BwdArgs {
    const float* rgb_fwd;
    const int32_t* nseg;
    const float* grad_rgb;
    float* grad_sigma;
    float* grad_sh;
    float thr;
    // per-leaf segment counts [2][L] from the training forward, or null (counted here)
    const uint32_t* leaf_count;
    // the forward's segment records (a == null: replay by traversal)
    SegRecords rec;
    // fused optimiser step (grad_* unused): RMSProp (rms) or Adam (adam, with
    // first moments m_*), second moments v_*; both null: plain adjoint
    float* m_sigma;
    float* m_sh;
    float* v_sigma;
    float* v_sh;
    const dot_rmsprop_params* rms;
    const dot_adam_params* adam;
    // rows of the bucket array, set by the adjoint before its emit kernels run
    uint32_t n_rows = 0;
};

// The optimiser updates below are evaluated without contraction into FMAs, so
// every kernel that applies them (the elementwise steps and the fused
// reductions) rounds the same way and their results agree bit for bit.
//
// RMSProp on one parameter: v = alpha v + (1 - alpha) g^2; theta -= lr g / (sqrt(v) + eps)
__device__ __forceinline__ void rmsprop_update(float& theta, float& v, float g, float lr, float alpha, float eps) {
#pragma clang fp contract(off)
    v = alpha * v + (1.f - alpha) * g * g;
    theta -= lr * g / (sqrtf(v) + eps);
}

// Adam (Kingma & Ba) on one parameter: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// theta -= lr (m / bc1) / (sqrt(v / bc2) + eps) with bc = 1 - b^t
__device__ __forceinline__ void adam_update(float& theta, float& m, float& v, float g, float lr, float b1, float b2,
                                            float eps, float bc1, float bc2) {
#pragma clang fp contract(off)
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    theta -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

hipError_t launch_render_fwd(const dot_tree& t, const RayBatch& rb, const FwdArgs& a, hipStream_t s);
hipError_t launch_render_bwd(const dot_tree& t, const RayBatch& rb, const BwdArgs& a, hipStream_t s);
// re-traversal adjoint with wave-level per-leaf sums before the float atomics
hipError_t launch_render_bwd_wave(const dot_tree& t, const RayBatch& rb, const BwdArgs& a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s, uint32_t* word = nullptr, int n_words = 1);
// training forward that recorded: queue the copy of its row total and overflow
// count for the adjoint (no effect when that cannot be set up: the adjoint then
// reads them back itself); the adjoint's lookup (null when there is none)
void note_forward(const dot_tree& t, const SegRecords& rec, const uint32_t* counts, int64_t n_rays, hipStream_t s);
const uint32_t* find_note(const dot_tree& t, const void* rec, const uint32_t* counts, int64_t n_rays, hipEvent_t* ev);
void drop_notes(const dot_tree& t);
hipError_t launch_encode_planes(int storage, const float* src, void* dst, int64_t rows, int src_cols,
                                int dst_stride, hipStream_t s);
hipError_t launch_decode_planes(int storage, const void* src, float* dst, int64_t rows, int dst_cols,
                                int src_stride, hipStream_t s);
hipError_t launch_adam(const dot_tree& t, const float* gs, const float* gh, float* ms, float* vs,
                       float* mh, float* vh, const dot_adam_params& p, hipStream_t s);
// Adam's bias corrections 1 - beta1^t and 1 - beta2^t (host, FP32)
inline void adam_bias_corrections(const dot_adam_params& p, float& bc1, float& bc2) {
    bc1 = 1.f - powf(p.beta1, (float)p.step);
    bc2 = 1.f - powf(p.beta2, (float)p.step);
}
// exclusive scan of n uint32 values; *tot receives the total (device); bsum
// needs scan_scratch_elems(n) elements
int64_t scan_scratch_elems(int64_t n);
hipError_t scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* bsum, uint32_t* tot, hipStream_t s);
// small arrays (one workgroup): exclusive scan of a + b into out and its total
// into *tot, also c = a + b, z = 0 and *w_dst = *w_src (when w_src); false
// (nothing launched) when n is too large for one workgroup
bool scan_u32_sum2(const uint32_t* a, const uint32_t* b, uint32_t* c, uint32_t* z, uint32_t* out, int64_t n,
                   uint32_t* tot, const uint32_t* w_src, uint32_t* w_dst, hipStream_t s, hipError_t* err);
hipError_t launch_rmsprop(const dot_tree& t, const float* gs, const float* gh, float* vs, float* vh,
                          const dot_rmsprop_params& p, hipStream_t s);
hipError_t launch_sigma_signal(const dot_tree& t, float* out, hipStream_t s);
hipError_t launch_mse(const float* pred, const float* target, const int64_t* idx, int64_t n, const double* gmul,
                      float* grad, double* loss, hipStream_t s);
size_t pixel_batch_workspace_bytes(int64_t n, int32_t W, int32_t H, int32_t n_cams);
hipError_t launch_pixel_batch(const int64_t* ids, int64_t n, int32_t W, int32_t H, int32_t n_cams, int32_t* cam_out,
                              int32_t* pix_out, int64_t* id_out, void* ws, hipStream_t s);
// device address of the no-allocation pixel batch's scratch on the current
// device (DOT_PIXEL_BATCH_SCRATCH_BYTES)
hipError_t pixel_batch_scratch(void** out);
hipError_t launch_stream_read(const void* buf, size_t bytes, float* sink, hipStream_t s);
size_t jobs_workspace_bytes(int n_jobs);
int launch_render_jobs(const dot_render_job* jobs, int n_jobs, void* ws, size_t ws_bytes, hipStream_t s);
int quantize_sh(dot_tree& t, int bits, hipStream_t s);
hipError_t launch_decode_palette(const dot_tree& t, float* dst, int64_t rows, int64_t row0, hipStream_t s);
int refine_tree(dot_tree& t, const float* signal, const dot_refine_params& p, dot_refine_stats* st,
                hipStream_t s);
// (re)build or drop t.links after the topology changed: built when t.links_on,
// the tree has internal nodes and n_leaves <= LINK_MAX_LEAVES; synchronises s
int update_links(dot_tree& t, hipStream_t s);

}  // namespace dot
