// C ABI of libdot: argument validation, tree upload/export, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dot_internal.h"

namespace dot {

// the gather probe's launcher (probe.hip)
hipError_t launch_gather_rows(const void* buf, int64_t n_rows_pow2, int64_t reads, float* sink, hipStream_t s);
hipError_t launch_atomic_count(uint32_t* counters, uint32_t n_counters, int64_t n, bool returning, hipStream_t s);

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return DOT_EHIP;
}

void* Alloc::get(size_t bytes) const {
    if (bytes == 0) bytes = 16;
    if (custom) return a.alloc(bytes, a.ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void Alloc::put(void* p) const {
    if (!p) return;
    if (custom)
        a.free(p, a.ctx);
    else
        (void)hipFree(p);
}

}  // namespace dot

// A kept block serves a request on its stream when it is large enough and not
// more than twice the request (or 64 KiB); a new block gets 1/8 headroom (requests that
// vary from step to step, like the adjoint's rows, then reuse it).
void* dot_tree::scratch_get(size_t bytes, hipStream_t s) const {
    if (bytes == 0) bytes = 16;
    size_t best = scratch_free.size();
    for (size_t i = 0; i < scratch_free.size(); ++i) {
        const ScratchBlock& b = scratch_free[i];
        if (b.s == s && b.cap >= bytes && b.cap <= std::max<size_t>(2 * bytes, 1 << 16) &&
            (best == scratch_free.size() || b.cap < scratch_free[best].cap))
            best = i;
    }
    if (best < scratch_free.size()) {
        const ScratchBlock b = scratch_free[best];
        scratch_free.erase(scratch_free.begin() + (std::ptrdiff_t)best);
        scratch_live.push_back(b);
        return b.p;
    }
    const size_t cap = (bytes + bytes / 8 + 4095) & ~(size_t)4095;
    void* p = alloc.get(cap);
    if (!p) return nullptr;
    scratch_live.push_back({p, cap, s});
    return p;
}

void dot_tree::scratch_put(void* p, hipStream_t s) const {
    if (!p) return;
    for (size_t i = 0; i < scratch_live.size(); ++i) {
        if (scratch_live[i].p != p) continue;
        ScratchBlock b = scratch_live[i];
        scratch_live.erase(scratch_live.begin() + (std::ptrdiff_t)i);
        b.s = s;
        scratch_free.push_back(b);
        // drop the oldest kept blocks beyond the limit (stream order still
        // covers them: the allocator's own reuse follows the caller's stream)
        while (scratch_free.size() > kScratchKept) {
            alloc.put(scratch_free.front().p);
            scratch_free.erase(scratch_free.begin());
        }
        return;
    }
    alloc.put(p);   // not a scratch block
}

void dot_tree::scratch_clear() const {
    for (const ScratchBlock& b : scratch_free) alloc.put(b.p);
    for (const ScratchBlock& b : scratch_live) alloc.put(b.p);
    scratch_free.clear();
    scratch_live.clear();
}

namespace dot {

// ---------------------------------------------------------------------------
// host-side validation of the canonical tree; fills leaf depths
// ---------------------------------------------------------------------------
static int validate_tree(const dot_tree_desc& d, std::vector<uint8_t>& depth, int& max_depth) {
    if (d.n_leaves < 1) return fail(DOT_EINVAL, "dot_build: n_leaves must be >= 1");
    if (d.n_internal < 0) return fail(DOT_EINVAL, "dot_build: n_internal must be >= 0");
    if (d.n_leaves > (int64_t)INT32_MAX || d.n_internal > (int64_t)INT32_MAX / 8)
        return fail(DOT_EINVAL, "dot_build: tree too large for 32-bit node indices");
    if (d.sh_degree < 0 || d.sh_degree > 3) return fail(DOT_EINVAL, "dot_build: sh_degree must be in 0..3");
    if (!(d.bbox_size > 0.f) || !std::isfinite(d.bbox_size))
        return fail(DOT_EINVAL, "dot_build: bbox_size must be positive and finite");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d.bbox_min[a])) return fail(DOT_EINVAL, "dot_build: bbox_min must be finite");
    if (!d.sigma || !d.sh) return fail(DOT_EINVAL, "dot_build: sigma and sh are required");
    depth.assign((size_t)d.n_leaves, 0);
    max_depth = 0;
    if (d.n_internal == 0) {
        if (d.n_leaves != 1) return fail(DOT_EINVAL, "dot_build: a tree with no internal node has exactly one leaf");
        return DOT_OK;
    }
    if (!d.child) return fail(DOT_EINVAL, "dot_build: child is required when n_internal > 0");
    struct Frame {
        int64_t node;
        int depth, oct;
    };
    std::vector<Frame> st;
    st.push_back({0, 0, 0});
    int64_t next_int = 1, next_leaf = 0;
    while (!st.empty()) {
        Frame& f = st.back();
        if (f.oct == 8) {
            st.pop_back();
            continue;
        }
        int64_t e = d.child[f.node * 8 + f.oct];
        int oct = f.oct++;
        int cd = f.depth + 1;
        if (cd > DOT_MAX_DEPTH)
            return fail(DOT_EINVAL, "dot_build: tree deeper than DOT_MAX_DEPTH (16)");
        if (e >= 0) {
            if (e >= d.n_internal)
                return fail(DOT_EINVAL, "dot_build: child[" + std::to_string(f.node) + "][" + std::to_string(oct) +
                                            "] = " + std::to_string(e) + " is out of range");
            if (e != next_int)
                return fail(DOT_EINVAL, "dot_build: internal node " + std::to_string(e) +
                                            " is referenced twice or not in depth-first pre-order (expected " +
                                            std::to_string(next_int) + ")");
            ++next_int;
            st.push_back({e, cd, 0});
        } else {
            int64_t l = -1 - e;
            if (l >= d.n_leaves)
                return fail(DOT_EINVAL, "dot_build: leaf id " + std::to_string(l) + " is out of range");
            if (l != next_leaf)
                return fail(DOT_EINVAL, "dot_build: leaf " + std::to_string(l) +
                                            " is referenced twice or leaves are not in depth-first order (expected " +
                                            std::to_string(next_leaf) + ")");
            depth[(size_t)l] = (uint8_t)cd;
            if (cd > max_depth) max_depth = cd;
            ++next_leaf;
        }
    }
    if (next_int != d.n_internal)
        return fail(DOT_EINVAL, "dot_build: " + std::to_string(d.n_internal - next_int) +
                                    " internal nodes are unreachable from the root");
    if (next_leaf != d.n_leaves)
        return fail(DOT_EINVAL, "dot_build: " + std::to_string(d.n_leaves - next_leaf) +
                                    " leaves are unreachable from the root");
    return DOT_OK;
}

// Copy a host FP32 matrix [rows][cols] into a device plane of the storage type
// with row stride `stride`, through a bounded staging buffer.
static int upload_plane(const Alloc& al, int storage, const float* host, void* dst, int64_t rows, int cols,
                        int stride, hipStream_t s) {
    const int64_t max_rows = std::max<int64_t>(1, (64ll << 20) / ((int64_t)cols * 4));
    int64_t chunk = std::min(rows, max_rows);
    float* stage = static_cast<float*>(al.get((size_t)chunk * cols * 4));
    if (!stage) return fail(DOT_ENOMEM, "dot_build: staging allocation failed");
    const int es = storage_bytes(storage);
    int rc = DOT_OK;
    for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
        int64_t n = std::min(chunk, rows - r0);
        hipError_t e = hipMemcpyAsync(stage, host + r0 * cols, (size_t)n * cols * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_encode_planes(storage, stage, static_cast<char*>(dst) + (size_t)r0 * stride * es, n, cols,
                                     stride, s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "dot_build: upload");
            break;
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (rc == DOT_OK && e != hipSuccess) rc = hip_fail(e, "dot_build: synchronise");
    al.put(stage);
    return rc;
}

static int download_plane(const Alloc& al, int storage, const void* src, float* host, int64_t rows, int cols,
                          int stride, hipStream_t s) {
    const int64_t max_rows = std::max<int64_t>(1, (64ll << 20) / ((int64_t)cols * 4));
    int64_t chunk = std::min(rows, max_rows);
    float* stage = static_cast<float*>(al.get((size_t)chunk * cols * 4));
    if (!stage) return fail(DOT_ENOMEM, "dot_export: staging allocation failed");
    const int es = storage_bytes(storage);
    int rc = DOT_OK;
    for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
        int64_t n = std::min(chunk, rows - r0);
        hipError_t e = launch_decode_planes(storage, static_cast<const char*>(src) + (size_t)r0 * stride * es, stage,
                                            n, cols, stride, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host + r0 * cols, stage, (size_t)n * cols * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "dot_export: download");
            break;
        }
    }
    al.put(stage);
    return rc;
}

static void release(dot_tree* t) {
    t->alloc.put(t->child);
    t->alloc.put(t->sigma);
    t->alloc.put(t->sh);
    t->alloc.put(t->leaf_depth);
    t->alloc.put(t->palette);
    t->alloc.put(t->links);
    t->links = nullptr;
    if (t->host_rb) (void)hipHostFree(t->host_rb);
    t->host_rb = nullptr;
    drop_notes(*t);
    t->scratch_clear();
    t->child = nullptr;
    t->sigma = nullptr;
    t->sh = nullptr;
    t->leaf_depth = nullptr;
    t->palette = nullptr;
}

// SH rows of a palette tree decoded to host FP32 [rows][nv], through staging
static int download_palette_sh(const dot_tree& t, float* host, hipStream_t s) {
    const int nv = 3 * (t.degree + 1) * (t.degree + 1);
    const int64_t rows = t.n_leaves;
    const int64_t chunk = std::min<int64_t>(rows, std::max<int64_t>(1, (64ll << 20) / ((int64_t)nv * 4)));
    float* stage = static_cast<float*>(t.alloc.get((size_t)chunk * nv * 4));
    if (!stage) return fail(DOT_ENOMEM, "dot_export: staging allocation failed");
    int rc = DOT_OK;
    for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
        const int64_t n = std::min(chunk, rows - r0);
        hipError_t e = launch_decode_palette(t, stage, n, r0, s);
        if (e == hipSuccess) e = hipMemcpyAsync(host + r0 * nv, stage, (size_t)n * nv * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "dot_export: download");
            break;
        }
    }
    t.alloc.put(stage);
    return rc;
}

static int make_batch(const dot_rays* r, RayBatch& rb, const char* who) {
    if (!r) return fail(DOT_EINVAL, std::string(who) + ": rays is NULL");
    std::memset(&rb, 0, sizeof(rb));
    rb.kind = r->kind;
    rb.n_cams = r->n_cams;
    rb.cams = r->cams;
    rb.width = r->width;
    rb.height = r->height;
    rb.n_rays = r->n_rays;
    rb.cam_idx = r->cam_idx;
    rb.pix_idx = r->pix_idx;
    rb.origins = r->origins;
    rb.dirs = r->dirs;
    if (r->kind == DOT_RAYS_CAMERAS) {
        if (r->n_cams < 0) return fail(DOT_EINVAL, std::string(who) + ": n_cams < 0");
        if (r->n_cams > 0 && (r->width <= 0 || r->height <= 0))
            return fail(DOT_EINVAL, std::string(who) + ": width and height must be positive");
        if (r->n_cams > 0 && !r->cams) return fail(DOT_EINVAL, std::string(who) + ": cams is NULL");
        int64_t tiles = r->n_cams > 0 ? (int64_t)r->n_cams * ((r->width + 7) / 8) * ((r->height + 7) / 8) : 0;
        rb.n_tiles = tiles;
        rb.n_rays = r->n_cams > 0 ? (int64_t)r->n_cams * r->width * r->height : 0;
    } else if (r->kind == DOT_RAYS_PIXELS || r->kind == DOT_RAYS_EXPLICIT) {
        if (r->n_rays < 0) return fail(DOT_EINVAL, std::string(who) + ": n_rays < 0");
        if (r->n_rays > 0) {
            if (r->kind == DOT_RAYS_PIXELS && (!r->cams || !r->cam_idx || !r->pix_idx || r->n_cams <= 0))
                return fail(DOT_EINVAL, std::string(who) + ": PIXELS rays need cams, cam_idx and pix_idx");
            if (r->kind == DOT_RAYS_EXPLICIT && (!r->origins || !r->dirs))
                return fail(DOT_EINVAL, std::string(who) + ": EXPLICIT rays need origins and dirs");
        }
        rb.n_tiles = (r->n_rays + 63) / 64;
    } else {
        return fail(DOT_EINVAL, std::string(who) + ": unknown ray kind " + std::to_string(r->kind));
    }
    if ((rb.n_tiles + 3) / 4 > (int64_t)INT32_MAX)
        return fail(DOT_EINVAL, std::string(who) + ": too many rays for one launch");
    return DOT_OK;
}

static int fill_opts(const dot_render_opts* o, float bg[3], float& thr, const char* who) {
    if (!o) {
        bg[0] = bg[1] = bg[2] = 1.f;
        thr = -std::log(1e-4f);
        return DOT_OK;
    }
    if (!(o->t_stop >= 0.f && o->t_stop < 1.f))
        return fail(DOT_EINVAL, std::string(who) + ": t_stop must be in [0, 1)");
    if (o->signal_mode != DOT_SIGNAL_MAX && o->signal_mode != DOT_SIGNAL_SUM)
        return fail(DOT_EINVAL, std::string(who) + ": unknown signal_mode");
    for (int a = 0; a < 3; ++a) bg[a] = o->bg[a];
    thr = o->t_stop > 0.f ? -std::log(o->t_stop) : __builtin_huge_valf();
    return DOT_OK;
}

// Adam's constants: decays in [0, 1), eps positive and finite, 1-based step
static int check_adam(const dot_adam_params& p, const char* who) {
    if (!(p.beta1 >= 0.f && p.beta1 < 1.f && p.beta2 >= 0.f && p.beta2 < 1.f))
        return fail(DOT_EINVAL, std::string(who) + ": beta1 and beta2 must be in [0, 1)");
    if (!(p.eps > 0.f && p.eps < __builtin_huge_valf()))
        return fail(DOT_EINVAL, std::string(who) + ": eps must be positive and finite");
    if (p.step < 1) return fail(DOT_EINVAL, std::string(who) + ": step must be >= 1");
    return DOT_OK;
}

}  // namespace dot

using namespace dot;

extern "C" {

const char* dot_last_error(void) { return g_err.c_str(); }

int dot_build(const dot_tree_desc* desc, int32_t storage, const dot_allocator* alloc, void* stream,
              dot_tree_t* out) {
    if (!out) return fail(DOT_EINVAL, "dot_build: out is NULL");
    *out = nullptr;
    if (!desc) return fail(DOT_EINVAL, "dot_build: desc is NULL");
    if (storage != DOT_F32 && storage != DOT_F16 && storage != DOT_BF16)
        return fail(DOT_EINVAL, "dot_build: unknown storage type " + std::to_string(storage));
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(DOT_EINVAL, "dot_build: allocator needs both alloc and free");
    std::vector<uint8_t> depth;
    int max_depth = 0;
    int rc = validate_tree(*desc, depth, max_depth);
    if (rc) return rc;

    dot_tree* t = new (std::nothrow) dot_tree();
    if (!t) return fail(DOT_ENOMEM, "dot_build: out of host memory");
    if (alloc) {
        t->alloc.a = *alloc;
        t->alloc.custom = true;
    }
    t->n_internal = desc->n_internal;
    t->n_leaves = desc->n_leaves;
    t->degree = desc->sh_degree;
    t->storage = storage;
    t->max_depth = max_depth;
    t->sh_stride = sh_stride_for(desc->sh_degree, storage);
    for (int a = 0; a < 3; ++a) t->bmin[a] = desc->bbox_min[a];
    t->size = desc->bbox_size;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int es = storage_bytes(storage);
    const int nv = 3 * (t->degree + 1) * (t->degree + 1);
    t->child = static_cast<int32_t*>(t->alloc.get((size_t)std::max<int64_t>(t->n_internal, 1) * 32));
    t->sigma = t->alloc.get((size_t)t->n_leaves * es);
    t->sh = t->alloc.get((size_t)t->n_leaves * t->sh_stride * es);
    t->leaf_depth = static_cast<uint8_t*>(t->alloc.get((size_t)t->n_leaves));
    if (!t->child || !t->sigma || !t->sh || !t->leaf_depth) {
        release(t);
        delete t;
        return fail(DOT_ENOMEM, "dot_build: device allocation failed");
    }
    hipError_t e = hipSuccess;
    if (t->n_internal > 0)
        e = hipMemcpyAsync(t->child, desc->child, (size_t)t->n_internal * 32, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t->leaf_depth, depth.data(), (size_t)t->n_leaves, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "dot_build: upload");
    } else {
        rc = upload_plane(t->alloc, storage, desc->sigma, t->sigma, t->n_leaves, 1, 1, s);
        if (!rc) rc = upload_plane(t->alloc, storage, desc->sh, t->sh, t->n_leaves, nv, t->sh_stride, s);
        if (!rc) rc = update_links(*t, s);
    }
    if (rc) {
        release(t);
        delete t;
        return rc;
    }
    *out = t;
    return DOT_OK;
}

int dot_free(dot_tree_t t) {
    if (!t) return DOT_OK;
    release(t);
    delete t;
    return DOT_OK;
}

int dot_tree_info(dot_tree_t t, dot_tree_info_t* out) {
    if (!t || !out) return fail(DOT_EINVAL, "dot_tree_info: NULL argument");
    out->n_internal = t->n_internal;
    out->n_leaves = t->n_leaves;
    out->sh_degree = t->degree;
    out->storage = t->storage;
    out->max_depth = t->max_depth;
    out->sh_stride = t->sh_stride;
    out->child = t->child;
    out->sigma = t->sigma;
    out->sh = t->sh;
    out->leaf_depth = t->leaf_depth;
    for (int a = 0; a < 3; ++a) out->bbox_min[a] = t->bmin[a];
    out->bbox_size = t->size;
    out->palette = t->palette;
    out->palette_bits = t->palette_bits;
    out->reserved = 0;
    out->links = t->links;
    return DOT_OK;
}

int dot_set_links(dot_tree_t t, int32_t enable, void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_set_links: tree is NULL");
    t->links_on = enable != 0;
    if (t->links_on && t->links) return DOT_OK;
    return update_links(*t, static_cast<hipStream_t>(stream));
}

int dot_render(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts, float* rgb_out, int32_t* nseg_out,
               float* signal_inout, void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_render: tree is NULL");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_render");
    if (rc) return rc;
    if (!rgb_out && rb.n_rays > 0) return fail(DOT_EINVAL, "dot_render: rgb_out is NULL");
    FwdArgs a{};
    rc = fill_opts(opts, a.bg, a.thr, "dot_render");
    if (rc) return rc;
    a.rgb = rgb_out;
    a.nseg = nseg_out;
    a.signal = signal_inout;
    a.signal_mode = opts ? opts->signal_mode : DOT_SIGNAL_MAX;
    hipError_t e = launch_render_fwd(*t, rb, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_render: launch");
    return DOT_OK;
}

size_t dot_render_train_records_bytes(int64_t n_rays, int32_t max_segments) {
    if (n_rays < 0 || max_segments < 1 || max_segments > SEG_CAP_MAX) return 0;
    return seg_records_bytes(n_rays, max_segments);
}

// the records view of a caller's buffer for a batch of n rays (validated)
static int records_for(const void* records, size_t bytes, int64_t n, SegRecords& out, const char* who) {
    out = SegRecords{};
    if (!records || n == 0) return DOT_OK;
    out = seg_records_view(const_cast<void*>(records), n, bytes);
    if (!out.a) return fail(DOT_EINVAL, std::string(who) + ": records buffer too small for one segment per ray");
    return DOT_OK;
}

int dot_render_train(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts, float* rgb_out,
                     int32_t* nseg_out, float* signal_inout, uint32_t* leaf_count_out, void* records,
                     size_t records_bytes, void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_render_train: tree is NULL");
    if (t->storage != DOT_F32) return fail(DOT_EUNSUPPORTED, "dot_render_train: only FP32 leaf storage is trainable");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_render_train");
    if (rc) return rc;
    if (!leaf_count_out) return fail(DOT_EINVAL, "dot_render_train: leaf_count_out is NULL");
    if (rb.n_rays > 0 && (!rgb_out || !nseg_out)) return fail(DOT_EINVAL, "dot_render_train: rgb_out and nseg_out are required");
    FwdArgs a{};
    rc = fill_opts(opts, a.bg, a.thr, "dot_render_train");
    if (rc) return rc;
    a.rgb = rgb_out;
    a.nseg = nseg_out;
    a.signal = signal_inout;
    a.signal_mode = opts ? opts->signal_mode : DOT_SIGNAL_MAX;
    a.leaf_count = leaf_count_out;
    a.leaf_rest = leaf_count_out + t->n_leaves;
    rc = records_for(records, records_bytes, rb.n_rays, a.rec, "dot_render_train");
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the records header's overflow count and row total start at zero
    hipError_t e = launch_fill_u32(leaf_count_out, 2 * t->n_leaves, s, a.rec.a ? a.rec.overflow : nullptr, 2);
    if (e == hipSuccess) e = launch_render_fwd(*t, rb, a, s);
    if (e != hipSuccess) return hip_fail(e, "dot_render_train: launch");
    if (a.rec.a && rb.n_rays > 0) note_forward(*t, a.rec, leaf_count_out, rb.n_rays, s);
    return DOT_OK;
}

int dot_accumulate_signal(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts, float* signal_inout,
                          void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_accumulate_signal: tree is NULL");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_accumulate_signal");
    if (rc) return rc;
    if (!signal_inout && t->n_leaves > 0) return fail(DOT_EINVAL, "dot_accumulate_signal: signal is NULL");
    FwdArgs a{};
    rc = fill_opts(opts, a.bg, a.thr, "dot_accumulate_signal");
    if (rc) return rc;
    a.signal = signal_inout;
    a.signal_mode = opts ? opts->signal_mode : DOT_SIGNAL_MAX;
    hipError_t e = launch_render_fwd(*t, rb, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_accumulate_signal: launch");
    return DOT_OK;
}

int dot_render_backward(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts, const float* rgb_fwd,
                        const int32_t* nseg, const float* grad_rgb, float* grad_sigma, float* grad_sh,
                        const uint32_t* leaf_count, const void* records, size_t records_bytes, void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_render_backward: tree is NULL");
    if (t->storage == DOT_PAL16)
        return fail(DOT_EUNSUPPORTED, "dot_render_backward: a palette-compressed tree is not differentiable");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_render_backward");
    if (rc) return rc;
    if (rb.n_rays > 0 && (!rgb_fwd || !nseg || !grad_rgb || !grad_sigma || !grad_sh))
        return fail(DOT_EINVAL, "dot_render_backward: rgb_fwd, nseg, grad_rgb, grad_sigma and grad_sh are required");
    BwdArgs a{};
    float bg[3];
    rc = fill_opts(opts, bg, a.thr, "dot_render_backward");
    if (rc) return rc;
    a.rgb_fwd = rgb_fwd;
    a.nseg = nseg;
    a.grad_rgb = grad_rgb;
    a.grad_sigma = grad_sigma;
    a.grad_sh = grad_sh;
    a.leaf_count = leaf_count;
    if (records && !leaf_count) return fail(DOT_EINVAL, "dot_render_backward: records need leaf_count");
    if (records && t->storage != DOT_F32)
        return fail(DOT_EINVAL, "dot_render_backward: records come from dot_render_train on an FP32 tree");
    rc = records_for(records, records_bytes, rb.n_rays, a.rec, "dot_render_backward");
    if (rc) return rc;
    hipError_t e = launch_render_bwd(*t, rb, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_render_backward: launch");
    return DOT_OK;
}

int dot_render_backward_atomic(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts, const float* rgb_fwd,
                               const int32_t* nseg, const float* grad_rgb, float* grad_sigma, float* grad_sh,
                               void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_render_backward_atomic: tree is NULL");
    if (t->storage == DOT_PAL16)
        return fail(DOT_EUNSUPPORTED, "dot_render_backward_atomic: a palette-compressed tree is not differentiable");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_render_backward_atomic");
    if (rc) return rc;
    if (rb.n_rays > 0 && (!rgb_fwd || !nseg || !grad_rgb || !grad_sigma || !grad_sh))
        return fail(DOT_EINVAL,
                    "dot_render_backward_atomic: rgb_fwd, nseg, grad_rgb, grad_sigma and grad_sh are required");
    BwdArgs a{};
    float bg[3];
    rc = fill_opts(opts, bg, a.thr, "dot_render_backward_atomic");
    if (rc) return rc;
    a.rgb_fwd = rgb_fwd;
    a.nseg = nseg;
    a.grad_rgb = grad_rgb;
    a.grad_sigma = grad_sigma;
    a.grad_sh = grad_sh;
    hipError_t e = launch_render_bwd_wave(*t, rb, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_render_backward_atomic: launch");
    return DOT_OK;
}

int dot_render_backward_rmsprop(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts,
                                const float* rgb_fwd, const int32_t* nseg, const float* grad_rgb, float* v_sigma,
                                float* v_sh, const dot_rmsprop_params* params, const uint32_t* leaf_count,
                                const void* records, size_t records_bytes, void* stream) {
    if (!t || !params) return fail(DOT_EINVAL, "dot_render_backward_rmsprop: NULL tree or params");
    if (t->storage != DOT_F32)
        return fail(DOT_EUNSUPPORTED, "dot_render_backward_rmsprop: only FP32 leaf storage is trainable");
    if (!(params->alpha >= 0.f && params->alpha < 1.f))
        return fail(DOT_EINVAL, "dot_render_backward_rmsprop: alpha must be in [0, 1)");
    if (!(params->eps > 0.f && params->eps < __builtin_huge_valf()))
        return fail(DOT_EINVAL, "dot_render_backward_rmsprop: eps must be positive and finite");
    if (!v_sigma || !v_sh) return fail(DOT_EINVAL, "dot_render_backward_rmsprop: square-average buffers are required");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_render_backward_rmsprop");
    if (rc) return rc;
    if (rb.n_rays > 0 && (!rgb_fwd || !nseg || !grad_rgb))
        return fail(DOT_EINVAL, "dot_render_backward_rmsprop: rgb_fwd, nseg and grad_rgb are required");
    BwdArgs a{};
    float bg[3];
    rc = fill_opts(opts, bg, a.thr, "dot_render_backward_rmsprop");
    if (rc) return rc;
    a.rgb_fwd = rgb_fwd;
    a.nseg = nseg;
    a.grad_rgb = grad_rgb;
    a.v_sigma = v_sigma;
    a.v_sh = v_sh;
    a.rms = params;
    a.leaf_count = leaf_count;
    if (records && !leaf_count) return fail(DOT_EINVAL, "dot_render_backward_rmsprop: records need leaf_count");
    rc = records_for(records, records_bytes, rb.n_rays, a.rec, "dot_render_backward_rmsprop");
    if (rc) return rc;
    hipError_t e = launch_render_bwd(*t, rb, a, static_cast<hipStream_t>(stream));
    if (e == hipErrorOutOfMemory) return fail(DOT_ENOMEM, "dot_render_backward_rmsprop: scratch allocation failed");
    if (e != hipSuccess) return hip_fail(e, "dot_render_backward_rmsprop: launch");
    return DOT_OK;
}

int dot_render_backward_adam(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts, const float* rgb_fwd,
                             const int32_t* nseg, const float* grad_rgb, float* m_sigma, float* v_sigma, float* m_sh,
                             float* v_sh, const dot_adam_params* params, const uint32_t* leaf_count,
                             const void* records, size_t records_bytes, void* stream) {
    if (!t || !params) return fail(DOT_EINVAL, "dot_render_backward_adam: NULL tree or params");
    if (t->storage != DOT_F32)
        return fail(DOT_EUNSUPPORTED, "dot_render_backward_adam: only FP32 leaf storage is trainable");
    if (int rc = check_adam(*params, "dot_render_backward_adam")) return rc;
    if (!m_sigma || !v_sigma || !m_sh || !v_sh)
        return fail(DOT_EINVAL, "dot_render_backward_adam: moment buffers are required");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_render_backward_adam");
    if (rc) return rc;
    if (rb.n_rays > 0 && (!rgb_fwd || !nseg || !grad_rgb))
        return fail(DOT_EINVAL, "dot_render_backward_adam: rgb_fwd, nseg and grad_rgb are required");
    BwdArgs a{};
    float bg[3];
    rc = fill_opts(opts, bg, a.thr, "dot_render_backward_adam");
    if (rc) return rc;
    a.rgb_fwd = rgb_fwd;
    a.nseg = nseg;
    a.grad_rgb = grad_rgb;
    a.m_sigma = m_sigma;
    a.v_sigma = v_sigma;
    a.m_sh = m_sh;
    a.v_sh = v_sh;
    a.adam = params;
    a.leaf_count = leaf_count;
    if (records && !leaf_count) return fail(DOT_EINVAL, "dot_render_backward_adam: records need leaf_count");
    rc = records_for(records, records_bytes, rb.n_rays, a.rec, "dot_render_backward_adam");
    if (rc) return rc;
    hipError_t e = launch_render_bwd(*t, rb, a, static_cast<hipStream_t>(stream));
    if (e == hipErrorOutOfMemory) return fail(DOT_ENOMEM, "dot_render_backward_adam: scratch allocation failed");
    if (e != hipSuccess) return hip_fail(e, "dot_render_backward_adam: launch");
    return DOT_OK;
}

int dot_render_stats(dot_tree_t t, const dot_rays* rays, const dot_render_opts* opts, int64_t counts[4],
                     void* stream) {
    if (!t || !counts) return fail(DOT_EINVAL, "dot_render_stats: NULL argument");
    RayBatch rb;
    int rc = make_batch(rays, rb, "dot_render_stats");
    if (rc) return rc;
    FwdArgs a{};
    rc = fill_opts(opts, a.bg, a.thr, "dot_render_stats");
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long* dev = static_cast<unsigned long long*>(t->alloc.get(4 * sizeof(unsigned long long)));
    if (!dev) return fail(DOT_ENOMEM, "dot_render_stats: allocation failed");
    unsigned long long host[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(dev, host, sizeof(host), hipMemcpyHostToDevice, s);
    a.stats = dev;
    if (e == hipSuccess) e = launch_render_fwd(*t, rb, a, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    t->alloc.put(dev);
    if (e != hipSuccess) return hip_fail(e, "dot_render_stats");
    for (int i = 0; i < 4; ++i) counts[i] = (int64_t)host[i];
    return DOT_OK;
}

int dot_adam_step(dot_tree_t t, const float* grad_sigma, const float* grad_sh, float* m_sigma, float* v_sigma,
                  float* m_sh, float* v_sh, const dot_adam_params* p, void* stream) {
    if (!t || !p) return fail(DOT_EINVAL, "dot_adam_step: NULL argument");
    if (t->storage != DOT_F32) return fail(DOT_EUNSUPPORTED, "dot_adam_step: only FP32 leaf storage is trainable");
    if (!grad_sigma || !grad_sh || !m_sigma || !v_sigma || !m_sh || !v_sh)
        return fail(DOT_EINVAL, "dot_adam_step: gradient and moment buffers are required");
    if (int rc = check_adam(*p, "dot_adam_step")) return rc;
    hipError_t e = launch_adam(*t, grad_sigma, grad_sh, m_sigma, v_sigma, m_sh, v_sh, *p,
                               static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_adam_step: launch");
    return DOT_OK;
}

int dot_rmsprop_step(dot_tree_t t, const float* grad_sigma, const float* grad_sh, float* v_sigma, float* v_sh,
                     const dot_rmsprop_params* p, void* stream) {
    if (!t || !p) return fail(DOT_EINVAL, "dot_rmsprop_step: NULL argument");
    if (t->storage != DOT_F32) return fail(DOT_EUNSUPPORTED, "dot_rmsprop_step: only FP32 leaf storage is trainable");
    if (!grad_sigma || !grad_sh || !v_sigma || !v_sh)
        return fail(DOT_EINVAL, "dot_rmsprop_step: gradient and square-average buffers are required");
    if (!(p->alpha >= 0.f && p->alpha < 1.f)) return fail(DOT_EINVAL, "dot_rmsprop_step: alpha must be in [0, 1)");
    if (!(p->eps > 0.f && p->eps < __builtin_huge_valf()))
        return fail(DOT_EINVAL, "dot_rmsprop_step: eps must be positive and finite");
    hipError_t e = launch_rmsprop(*t, grad_sigma, grad_sh, v_sigma, v_sh, *p, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_rmsprop_step: launch");
    return DOT_OK;
}

int dot_sigma_signal(dot_tree_t t, float* signal_out, void* stream) {
    if (!t || !signal_out) return fail(DOT_EINVAL, "dot_sigma_signal: NULL argument");
    hipError_t e = launch_sigma_signal(*t, signal_out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_sigma_signal: launch");
    return DOT_OK;
}

size_t dot_pixel_batch_workspace(int64_t n_rays, int32_t width, int32_t height, int32_t n_cams) {
    if (n_rays < 0 || width <= 0 || height <= 0 || n_cams <= 0) return 0;
    return pixel_batch_workspace_bytes(n_rays, width, height, n_cams);
}

int dot_pixel_batch(const int64_t* ray_ids, int64_t n_rays, int32_t width, int32_t height, int32_t n_cams,
                    int32_t* cam_idx_out, int32_t* pix_idx_out, int64_t* ray_ids_out, void* workspace,
                    size_t workspace_bytes, void* stream) {
    if (n_rays < 0) return fail(DOT_EINVAL, "dot_pixel_batch: n_rays < 0");
    if (width <= 0 || height <= 0 || n_cams <= 0)
        return fail(DOT_EINVAL, "dot_pixel_batch: width, height and n_cams must be positive");
    if ((int64_t)width * height > INT32_MAX) return fail(DOT_EINVAL, "dot_pixel_batch: image larger than 2^31 pixels");
    if (n_rays > (int64_t)UINT32_MAX) return fail(DOT_EINVAL, "dot_pixel_batch: more than 2^32 - 1 rays");
    if (n_rays == 0) return DOT_OK;
    if (!ray_ids || !cam_idx_out || !pix_idx_out || !workspace)
        return fail(DOT_EINVAL, "dot_pixel_batch: NULL ids, outputs or workspace");
    if (workspace_bytes < pixel_batch_workspace_bytes(n_rays, width, height, n_cams))
        return fail(DOT_EINVAL, "dot_pixel_batch: workspace too small");
    hipError_t e = launch_pixel_batch(ray_ids, n_rays, width, height, n_cams, cam_idx_out, pix_idx_out, ray_ids_out,
                                      workspace, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_pixel_batch: launch");
    return DOT_OK;
}

int dot_pixel_batch_noalloc(const int64_t* ray_ids, int64_t n_rays, int32_t width, int32_t height, int32_t n_cams,
                            int32_t* cam_idx_out, int32_t* pix_idx_out, int64_t* ray_ids_out, void* stream) {
    if (n_rays < 0) return fail(DOT_EINVAL, "dot_pixel_batch_noalloc: n_rays < 0");
    if (width <= 0 || height <= 0 || n_cams <= 0)
        return fail(DOT_EINVAL, "dot_pixel_batch_noalloc: width, height and n_cams must be positive");
    if ((int64_t)width * height > INT32_MAX)
        return fail(DOT_EINVAL, "dot_pixel_batch_noalloc: image larger than 2^31 pixels");
    if (n_rays > (int64_t)UINT32_MAX) return fail(DOT_EINVAL, "dot_pixel_batch_noalloc: more than 2^32 - 1 rays");
    if (n_rays == 0) return DOT_OK;
    if (!ray_ids || !cam_idx_out || !pix_idx_out) return fail(DOT_EINVAL, "dot_pixel_batch_noalloc: NULL ids or outputs");
    const size_t need = pixel_batch_workspace_bytes(n_rays, width, height, n_cams);
    if (need > (size_t)DOT_PIXEL_BATCH_SCRATCH_BYTES)
        return fail(DOT_EINVAL, "dot_pixel_batch_noalloc: the batch needs " + std::to_string(need) +
                                    " bytes of scratch, more than the " +
                                    std::to_string((size_t)DOT_PIXEL_BATCH_SCRATCH_BYTES) + " it holds");
    void* ws = nullptr;
    hipError_t e = pixel_batch_scratch(&ws);
    if (e != hipSuccess) return hip_fail(e, "dot_pixel_batch_noalloc: scratch address");
    e = launch_pixel_batch(ray_ids, n_rays, width, height, n_cams, cam_idx_out, pix_idx_out, ray_ids_out, ws,
                           static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_pixel_batch_noalloc: launch");
    return DOT_OK;
}

int dot_mse_loss(const float* pred, const float* target, const int64_t* target_idx, int64_t n_rays,
                 float* grad_rgb_out, double* loss_out, void* stream) {
    if (n_rays < 0) return fail(DOT_EINVAL, "dot_mse_loss: n_rays < 0");
    if (n_rays > 0 && (!pred || !target)) return fail(DOT_EINVAL, "dot_mse_loss: NULL prediction or target");
    hipError_t e = launch_mse(pred, target, target_idx, n_rays, nullptr, grad_rgb_out, loss_out,
                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_mse_loss: launch");
    return DOT_OK;
}

int dot_mse_grad(const float* pred, const float* target, const int64_t* target_idx, int64_t n_rays,
                 const double* scale, float* grad_rgb_out, void* stream) {
    if (n_rays < 0) return fail(DOT_EINVAL, "dot_mse_grad: n_rays < 0");
    if (n_rays > 0 && (!pred || !target || !grad_rgb_out))
        return fail(DOT_EINVAL, "dot_mse_grad: NULL prediction, target or gradient");
    if (n_rays == 0) return DOT_OK;
    hipError_t e = launch_mse(pred, target, target_idx, n_rays, scale, grad_rgb_out, nullptr,
                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_mse_grad: launch");
    return DOT_OK;
}

int dot_export(dot_tree_t t, int32_t* child, float* sigma, float* sh, uint8_t* leaf_depth, void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_export: tree is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (child && t->n_internal > 0)
        e = hipMemcpyAsync(child, t->child, (size_t)t->n_internal * 32, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && leaf_depth)
        e = hipMemcpyAsync(leaf_depth, t->leaf_depth, (size_t)t->n_leaves, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "dot_export");
    int nv = 3 * (t->degree + 1) * (t->degree + 1);
    int rc = DOT_OK;
    const int sst = t->storage == DOT_PAL16 ? DOT_F16 : t->storage;
    if (sigma) rc = download_plane(t->alloc, sst, t->sigma, sigma, t->n_leaves, 1, 1, s);
    if (!rc && sh) {
        if (t->storage == DOT_PAL16)
            rc = download_palette_sh(*t, sh, s);
        else
            rc = download_plane(t->alloc, t->storage, t->sh, sh, t->n_leaves, nv, t->sh_stride, s);
    }
    return rc;
}

int dot_refine(dot_tree_t t, const float* signal, const dot_refine_params* p, dot_refine_stats* stats,
               void* stream) {
    if (!t || !p) return fail(DOT_EINVAL, "dot_refine: NULL argument");
    if (!signal) return fail(DOT_EINVAL, "dot_refine: signal is NULL");
    if (t->storage == DOT_PAL16)
        return fail(DOT_EUNSUPPORTED, "dot_refine: a palette-compressed tree cannot be refined");
    if (!(p->sample_frac >= 0.f && p->sample_frac <= 1.f))
        return fail(DOT_EINVAL, "dot_refine: sample_frac must be in [0, 1]");
    if (p->max_depth < 0 || p->max_depth > DOT_MAX_DEPTH)
        return fail(DOT_EINVAL, "dot_refine: max_depth must be in 0..DOT_MAX_DEPTH");
    if (!std::isfinite(p->prune_tau)) return fail(DOT_EINVAL, "dot_refine: prune_tau must be finite");
    return refine_tree(*t, signal, *p, stats, static_cast<hipStream_t>(stream));
}

int dot_quantize_sh(dot_tree_t t, int32_t bits, void* stream) {
    if (!t) return fail(DOT_EINVAL, "dot_quantize_sh: tree is NULL");
    if (bits < 1 || bits > 16) return fail(DOT_EINVAL, "dot_quantize_sh: bits must be in 1..16");
    if (t->storage == DOT_PAL16) return fail(DOT_EINVAL, "dot_quantize_sh: the tree is already palette-compressed");
    return quantize_sh(*t, bits, static_cast<hipStream_t>(stream));
}

int dot_stream_read(const void* buf, size_t bytes, float* sink, void* stream) {
    if (bytes > 0 && (!buf || !sink)) return fail(DOT_EINVAL, "dot_stream_read: NULL buffer or sink");
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return fail(DOT_EINVAL, "dot_stream_read: buffer not 16-byte aligned");
    hipError_t e = launch_stream_read(buf, bytes, sink, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_stream_read: launch");
    return DOT_OK;
}

int dot_gather_rows(const void* buf, int64_t n_rows, int64_t reads, float* sink, void* stream) {
    if (n_rows <= 0 || (n_rows & (n_rows - 1)) != 0) return fail(DOT_EINVAL, "dot_gather_rows: n_rows must be a power of two");
    if (!buf || !sink) return fail(DOT_EINVAL, "dot_gather_rows: NULL buffer or sink");
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return fail(DOT_EINVAL, "dot_gather_rows: buffer not 16-byte aligned");
    const hipError_t e = dot::launch_gather_rows(buf, n_rows, reads, sink, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_gather_rows: launch");
    return DOT_OK;
}

int dot_atomic_count(uint32_t* counters, uint32_t n_counters, int64_t n, int returning, void* stream) {
    if (n < 0) return fail(DOT_EINVAL, "dot_atomic_count: n < 0");
    if (n > 0 && (!counters || n_counters == 0)) return fail(DOT_EINVAL, "dot_atomic_count: NULL or no counters");
    const hipError_t e = dot::launch_atomic_count(counters, n_counters, n, returning != 0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dot_atomic_count: launch");
    return DOT_OK;
}

size_t dot_render_jobs_workspace(int32_t n_jobs) { return jobs_workspace_bytes(n_jobs < 0 ? 0 : n_jobs); }

int dot_render_jobs(const dot_render_job* jobs, int32_t n_jobs, void* workspace, size_t workspace_bytes,
                    void* stream) {
    if (n_jobs < 0) return fail(DOT_EINVAL, "dot_render_jobs: n_jobs < 0");
    if (n_jobs == 0) return DOT_OK;
    if (!jobs || !workspace) return fail(DOT_EINVAL, "dot_render_jobs: jobs and workspace are required");
    return launch_render_jobs(jobs, n_jobs, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"
