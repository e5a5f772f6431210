/*
 * dot.h -- C ABI of the MI355X (gfx950) octree volume renderer of the
 * Dynamic PlenOctree method (DOT, arXiv 2307.15333).
 *
 * The library renders, differentiates and refines a sparse octree whose
 * leaves hold a density sigma and real spherical-harmonic (SH) colour
 * coefficients.  Every call is plain C: host or device pointers and sizes.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  - Return value: DOT_OK (0) or a negative DOT_E* code; the message of the
 *    last failure on the calling thread is returned by dot_last_error().
 *    No C++ exception crosses this interface.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  All
 *    device work is enqueued asynchronously on it unless stated otherwise.
 *  - Ownership: buffers passed in by the caller stay the caller's; the
 *    library never frees them.  Tree planes are owned by the dot_tree_t
 *    handle and released by dot_free.
 *  - Device pointers passed in must be valid for the stated size; kernels do
 *    not re-validate individual values (trees are validated at dot_build).
 *
 * Octree (canonical host form, accepted by dot_build)
 * ---------------------------------------------------
 *  Root cube [bbox_min, bbox_min + bbox_size]^3.  child is int32
 *  [n_internal][8]; octant o = x | y<<1 | z<<2 (bit set = upper half of that
 *  axis); an entry >= 0 is an internal node, an entry < 0 is leaf (-1-entry).
 *  Node 0 is the root; a tree whose root is a leaf has n_internal = 0 and
 *  n_leaves = 1.  Internal nodes are numbered in depth-first pre-order and
 *  leaves in depth-first order (children visited in octant order), so leaves
 *  are in Morton order.  Leaf depth <= DOT_MAX_DEPTH.
 *  Leaf payload (Sec. 3, "Preliminaries"; Sec. 4.1 stores 16 SH coefficients
 *  per channel plus a density): sigma[L] and sh[L][3][K] with
 *  K = (sh_degree+1)^2, real orthonormal SH with the Condon-Shortley phase,
 *  index k = l^2 + l + m.
 */
#ifndef DOT_H_
#define DOT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DOT_OK = 0,
    DOT_EINVAL = -1,       /* malformed argument or tree */
    DOT_ENOMEM = -2,       /* allocation failed */
    DOT_EHIP = -3,         /* HIP runtime error (message from hipGetErrorString) */
    DOT_EUNSUPPORTED = -4, /* valid request the library does not support (e.g. training reduced-precision leaves) */
    DOT_EBUSY = -5         /* a serving queue is full: retry once one of its jobs has completed */
};

/* leaf storage precision of the sigma and SH planes; arithmetic is FP32.
 * DOT_PAL16 (made only by dot_quantize_sh): FP16 sigma, a uint16 palette index
 * per leaf and an FP16 palette of SH rows. */
enum { DOT_F32 = 0, DOT_F16 = 1, DOT_BF16 = 2, DOT_PAL16 = 3 };

/* how rays are given */
enum {
    DOT_RAYS_CAMERAS = 0,  /* every pixel of n_cams cameras of width x height */
    DOT_RAYS_PIXELS = 1,   /* an explicit list of (camera, pixel) pairs */
    DOT_RAYS_EXPLICIT = 2  /* explicit origins and directions */
};

/* per-leaf training signal aggregate over rays (Sec. 3.1) */
enum { DOT_SIGNAL_MAX = 0, DOT_SIGNAL_SUM = 1 };

#define DOT_MAX_DEPTH 16

typedef struct dot_tree *dot_tree_t;

/* Device-memory allocator used for every allocation a tree makes (its planes,
 * refinement scratch, upload staging, the adjoint's buckets).  NULL =
 * hipMalloc/hipFree.  alloc returns NULL on failure (the call then fails with
 * DOT_ENOMEM).  A block may be freed while work queued on the call's stream
 * still uses it (stream-ordered reuse, as a caching allocator on that stream
 * provides); the adjoint's scratch is kept by the tree between calls on one
 * stream and only goes back to the allocator beyond a small number of blocks
 * or at dot_free. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} dot_allocator;

typedef struct {
    int64_t n_internal;
    int64_t n_leaves;
    int32_t sh_degree;      /* 0..3 */
    int32_t reserved;
    const int32_t *child;   /* host [n_internal][8] */
    const float *sigma;     /* host [n_leaves] raw density (pre-activation) */
    const float *sh;        /* host [n_leaves][3][K] */
    float bbox_min[3];
    float bbox_size;
} dot_tree_desc;

/* Pinhole camera: c2w is the row-major 3x4 [R | t] camera-to-world matrix
 * (camera axes x right, y down, z forward).  The ray of pixel (u, v) has
 * origin t and direction normalize(R ((u+0.5-cx)/fx, (v+0.5-cy)/fy, 1)). */
typedef struct {
    float c2w[12];
    float fx, fy, cx, cy;
    int32_t width, height;
} dot_camera;

/* Ray batch.  Ray order: CAMERAS = camera-major, then row-major pixels
 * (ray id = cam * H * W + v * W + u); PIXELS / EXPLICIT = list order. */
typedef struct {
    int32_t kind;               /* DOT_RAYS_* */
    int32_t n_cams;             /* CAMERAS, PIXELS */
    const dot_camera *cams;     /* DEVICE [n_cams] (CAMERAS, PIXELS) */
    int32_t width, height;      /* CAMERAS: image size shared by all cameras */
    int64_t n_rays;             /* PIXELS, EXPLICIT */
    const int32_t *cam_idx;     /* DEVICE [n_rays] (PIXELS) */
    const int32_t *pix_idx;     /* DEVICE [n_rays] (PIXELS): v * width + u */
    const float *origins;       /* DEVICE [n_rays][3] (EXPLICIT) */
    const float *dirs;          /* DEVICE [n_rays][3] (EXPLICIT), normalised inside */
} dot_rays;

typedef struct {
    float bg[3];            /* background colour added with the remaining transmittance */
    float t_stop;           /* stop a ray once exp(-S) < t_stop; 0 disables */
    int32_t signal_mode;    /* DOT_SIGNAL_MAX or DOT_SIGNAL_SUM */
    int32_t reserved;
} dot_render_opts;

typedef struct {
    int64_t n_internal, n_leaves;
    int32_t sh_degree, storage;   /* storage: DOT_F32/F16/BF16 */
    int32_t max_depth;            /* deepest leaf */
    int32_t sh_stride;            /* elements per leaf row of the SH plane (>= 3K, padded) */
    void *child;                  /* device int32 [n_internal][8] */
    void *sigma;                  /* device [n_leaves] in the storage type */
    void *sh;                     /* device [n_leaves][sh_stride]; row = [3][K] then padding */
    void *leaf_depth;             /* device uint8 [n_leaves] */
    float bbox_min[3], bbox_size;
    void *palette;                /* DOT_PAL16: device FP16 [2^palette_bits][sh_stride]; else NULL.
                                     sh is then the uint16 index plane [n_leaves] */
    int32_t palette_bits, reserved;
    void *links;                  /* device uint32 [n_leaves][6] face-neighbour links, or NULL (dot_set_links) */
} dot_tree_info_t;

/*
 * dot_build -- validate a canonical host tree and upload it.
 *  storage: DOT_F32 copies the planes; DOT_F16 / DOT_BF16 round each value to
 *  nearest-even on the device.  The host arrays are read during the call only.
 *  Errors: DOT_EINVAL for an out-of-range child entry, a node or leaf
 *  referenced twice or never, a child numbered before its parent (cycle or
 *  non pre-order), leaves not in DFS order, depth > DOT_MAX_DEPTH, a bad
 *  degree, storage or box; DOT_ENOMEM / DOT_EHIP from the device.
 *  The call synchronises `stream` before returning.
 */
int dot_build(const dot_tree_desc *desc, int32_t storage, const dot_allocator *alloc, void *stream,
              dot_tree_t *out);

/* dot_free -- release a tree and all device memory it owns (NULL is a no-op). */
int dot_free(dot_tree_t tree);

/* dot_tree_info -- sizes and device pointers of the tree's planes.  Pointers
 * stay valid until the next dot_refine or dot_free on the tree (links: also
 * dot_set_links). */
int dot_tree_info(dot_tree_t tree, dot_tree_info_t *out);

/*
 * dot_set_links -- keep (enable != 0) or drop (enable = 0) the tree's
 *  face-neighbour links.  They are an acceleration structure of the leaf walk,
 *  not part of the method: six uint32 per leaf (24 B of device memory per
 *  leaf) naming, for each face, the internal node of the same depth or the
 *  leaf of the same or a shallower depth across it (or the outside of the
 *  root cube).  With them a ray finds its next leaf from one link read issued
 *  together with the current leaf's data, descending only into a finer
 *  neighbour, instead of re-descending the child array from the deepest
 *  common ancestor.  The leaves visited and the segment lengths, hence every
 *  rendered value, gradient and signal, are the same either way.
 *  Links are built by dot_build and rebuilt by dot_refine while enabled; a
 *  tree of more than 2^27 - 1 leaves, or a root leaf, walks without them.
 *  Synchronises `stream`.  Errors: DOT_EINVAL on a NULL tree; DOT_ENOMEM /
 *  DOT_EHIP while building (the tree then walks without links).  dot_refine
 *  returns these codes too when the refined tree's links cannot be built; the
 *  refinement itself is then complete.
 */
int dot_set_links(dot_tree_t tree, int32_t enable, void *stream);

/*
 * dot_render -- forward volume rendering (Sec. 3 "Preliminaries", Eq. 1-2).
 *  For each ray: clip to the root cube, visit the leaves it crosses front to
 *  back with exact segment lengths delta_i, and composite
 *      C = sum_i T_i (1 - exp(-sigma^_i delta_i)) c_i + T_end bg,
 *      T_i = exp(-sum_{j<i} sigma^_j delta_j),  sigma^ = max(sigma, 0),
 *      c_i = sigmoid(sum_k sh_i[ch][k] Y_k(d))  per channel.
 *  A ray stops after the segment that drives exp(-S) below t_stop.
 *  rgb_out:   DEVICE float [n][3], required.
 *  nseg_out:  DEVICE int32 [n] or NULL: segments visited (delta > 0), the
 *             count dot_render_backward replays.
 *  signal_inout: DEVICE float [n_leaves] or NULL: fused training signal
 *             (Sec. 3.1, Alg. 1 "Q, pred <- render(rays)"): per leaf the max
 *             (DOT_SIGNAL_MAX) or sum (DOT_SIGNAL_SUM) over rays of the ray
 *             weight w_i = T_i (1 - exp(-sigma^_i delta_i)), accumulated into
 *             the existing values (MAX expects non-negative initial values).
 *  Errors: DOT_EINVAL on NULL tree/rays/rgb_out or an inconsistent ray batch.
 */
int dot_render(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts, float *rgb_out,
               int32_t *nseg_out, float *signal_inout, void *stream);

/*
 * dot_render_train -- the forward pass of a training step: dot_render with
 *  nseg_out required, plus leaf_count_out: DEVICE uint32 [2][n_leaves],
 *  overwritten with, per leaf, the number of this batch's segments whose
 *  leaf has sigma > 0 -- the segments whose gradient rows the adjoint emits --
 *  split into [0][l] the segments recorded (below) and [1][l] the others
 *  (all of them when records is NULL).  Given to dot_render_backward /
 *  dot_render_backward_rmsprop with the same tree, rays and opts, it lets the
 *  adjoint skip its own counting traversal.
 *  records: DEVICE buffer or NULL.  When given, the forward also records each
 *  ray's first `max_segments` segments whose leaf has sigma > 0 (leaf, delta,
 *  optical depth, colour and the slot its gradient row will take in the
 *  leaf's bucket, reserved here; 28 bytes each), max_segments being the
 *  largest count for which dot_render_train_records_bytes(n_rays,
 *  max_segments) fits in records_bytes (at most 1024).  The adjoint then
 *  replays them instead of traversing the tree and fetching the leaves again,
 *  without atomics, and re-traverses only the rays that had more, for their
 *  remaining segments.  The layout is private to the library; the buffer
 *  stays the caller's.
 *  FP32 storage only (DOT_EUNSUPPORTED otherwise); DOT_EINVAL on a records
 *  buffer too small for one segment per ray.
 */
size_t dot_render_train_records_bytes(int64_t n_rays, int32_t max_segments);
int dot_render_train(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts, float *rgb_out,
                     int32_t *nseg_out, float *signal_inout, uint32_t *leaf_count_out, void *records,
                     size_t records_bytes, void *stream);

/*
 * dot_accumulate_signal -- the signal pass alone (same traversal and weights as
 * dot_render, no colour output): signal_inout DEVICE float [n_leaves], required.
 */
int dot_accumulate_signal(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts,
                          float *signal_inout, void *stream);

/*
 * dot_render_backward -- adjoint of dot_render for a loss L(C) (Sec. 3: the
 *  renderer is fully differentiable and optimised under an MSE loss).  Each ray
 *  is re-traversed for nseg[r] segments; with P_i = sum_{j<=i} w_j c_j,
 *      dL/dsigma_i += [sigma_i > 0] delta_i sum_ch g_ch (T_{i+1} c_ch - (C_ch - P_i,ch))
 *      dL/dsh_i[ch][k] += g_ch w_i c_ch (1 - c_ch) Y_k(d)
 *  where g = grad_rgb[r] = dL/dC and C = rgb_fwd[r] (the forward output).
 *  rgb_fwd, grad_rgb: DEVICE float [n][3]; nseg: DEVICE int32 [n] from dot_render
 *  with the same tree, rays and opts.  grad_sigma: DEVICE float [n_leaves],
 *  grad_sh: DEVICE float [n_leaves][3][K] (dense); both accumulated into (+=),
 *  the caller zeroes them.  Contributions are grouped into per-leaf buckets
 *  (a counting pass, a prefix scan, a pass that writes each segment's
 *  compact gradient row -- dsigma, g_ch w c_ch (1 - c_ch) and the ray
 *  direction -- into its leaf's bucket, then per-leaf sums that expand the SH
 *  outer product), which needs device scratch of 32 B (16 B at degree 0) per
 *  contributing segment from the tree's allocator.  Sizing it needs the
 *  batch's row total on the host: with the records of a dot_render_train call
 *  that recorded (matched by its records and counts buffers, among the tree's
 *  last four such calls) the call waits only for that forward's copy of its
 *  row total, queued behind it; otherwise it synchronises `stream` once after
 *  its own scan (the words come back through pinned host buffers the tree
 *  allocates on first use and keeps until dot_free).  Scratch blocks return
 *  to a per-tree cache for the next call on the same stream (at most twelve
 *  blocks, freed through the allocator beyond that and at dot_free), so the
 *  adjoints of one tree must not run concurrently; beyond 8 GiB of
 *  scratch, or if it cannot be allocated, the terms go straight to the
 *  arrays with FP32 atomics; the same happens when n_rays times the tree's
 *  bound on segments per ray (3 * 2^max_depth + 64) reaches 2^32, since
 *  bucket offsets are 32-bit.  Summation order, hence the last bits, depends
 *  on scheduling.  leaf_count: NULL, or the [2][n_leaves] counts
 *  dot_render_train wrote for the same tree, rays and opts (the counting
 *  traversal is then skipped; counts or records from another batch give wrong
 *  gradients, never an access outside the buffers).  records: NULL, or the
 *  records that same dot_render_train call wrote (requires leaf_count;
 *  `records_bytes` as given to it).  leaf_count without records (also after a
 *  forward that recorded) re-traverses every ray and uses the two counts
 *  summed.
 */
int dot_render_backward(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts,
                        const float *rgb_fwd, const int32_t *nseg, const float *grad_rgb,
                        float *grad_sigma, float *grad_sh, const uint32_t *leaf_count, const void *records,
                        size_t records_bytes, void *stream);

/*
 * dot_render_backward_atomic -- the same adjoint (Sec. 3: the renderer is
 *  fully differentiable) by re-traversal alone: each ray walks its nseg[r]
 *  segments again, keeping only the prefix colour sum against the forward's
 *  colour (no per-segment state), and at every step the lanes of a wavefront
 *  that composite the same leaf sum their 1 + 3K terms across lanes (a
 *  segmented reduction over runs of equal leaf id in lane order) before one
 *  FP32 atomic per run and term into grad_sigma / grad_sh (accumulated, +=;
 *  the caller zeroes them).  Needs no scratch and never synchronises the
 *  stream, so it can be captured in a graph; arguments, layout and errors as
 *  dot_render_backward without leaf_count and records.  Summation order, hence
 *  the last bits, depends on scheduling.
 */
int dot_render_backward_atomic(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts,
                               const float *rgb_fwd, const int32_t *nseg, const float *grad_rgb,
                               float *grad_sigma, float *grad_sh, void *stream);

typedef struct {
    float prune_tau;     /* prune selection: signal <= tau (prune_le) or < tau */
    float sample_frac;   /* k = floor(sample_frac * n_leaves) leaves to subdivide */
    int32_t prune_le;
    int32_t max_depth;   /* only leaves shallower than this are subdivided */
    int32_t recursive;   /* 1: repeat merging up the hierarchy (the paper's "(R)" option) */
    int32_t reinit;      /* 1: new leaves start at sigma = 0, SH = 0 instead of the fused values
                            (the paper's ablation without feature fusion, App. C.1) */
} dot_refine_params;

typedef struct {
    int64_t leaves_before, leaves_after, internal_after;
    int64_t merged;      /* internal nodes turned into leaves */
    int64_t subdivided;  /* leaves turned into internal nodes */
} dot_refine_stats;

/*
 * dot_refine -- one refinement of the tree from a per-leaf signal (Sec. 3.2,
 *  Alg. 1: pruning then sampling from the same signal).
 *   prune (Eq. 3): an internal node whose 8 children are all leaves and all
 *     selected becomes a leaf holding the mean of the children's raw sigma and
 *     SH, rounded once to the storage type;
 *   recursive pruning (Sec. 3.2, Alg. 1 with rec): merging repeats, a merged
 *     node's signal being the max of its children's, until no group is
 *     selected -- every node whose subtree leaves are all selected becomes a
 *     leaf; its value is Eq. 3 applied level by level (mean of the 8
 *     children's values, each rounded to the storage type when formed);
 *   sample (Eq. 4): among leaves not selected for pruning and shallower than
 *     max_depth, the k with the largest signal (ties: lower leaf index first)
 *     become internal nodes whose 8 children copy the parent's values.
 *  The new tree is canonical (DFS numbering), so its topology is unique.
 *  signal: DEVICE float [n_leaves] (not modified).  The tree's planes are
 *  replaced; earlier dot_tree_info pointers become invalid.  stats may be NULL.
 *  Synchronises `stream` once to size the new planes.
 */
int dot_refine(dot_tree_t tree, const float *signal, const dot_refine_params *params,
               dot_refine_stats *stats, void *stream);

typedef struct {
    float lr_sigma, lr_sh;     /* learning rates (the paper's RMSProp uses 0.1 / 0.01) */
    float beta1, beta2, eps;
    int32_t step;              /* 1-based step number for bias correction */
} dot_adam_params;

/*
 * dot_adam_step -- one Adam update of the tree's sigma and SH planes in place
 *  (FP32 storage only).  grad_*: DEVICE float, dense layouts as in
 *  dot_render_backward; m_* / v_*: DEVICE float moments of the same shapes,
 *  zero-initialised by the caller before step 1.
 *  Errors: DOT_EUNSUPPORTED for FP16/BF16 storage; DOT_EINVAL for beta1 or
 *  beta2 outside [0, 1), eps not positive and finite, or step < 1.
 */
int dot_adam_step(dot_tree_t tree, const float *grad_sigma, const float *grad_sh, float *m_sigma,
                  float *v_sigma, float *m_sh, float *v_sh, const dot_adam_params *params,
                  void *stream);

typedef struct {
    float lr_sigma, lr_sh;     /* learning rates (the paper: 0.1 for sigma, 0.01 for SH, Sec. 4.1) */
    float alpha, eps;          /* square-average decay in [0, 1) and denominator term (> 0, finite) */
} dot_rmsprop_params;

/*
 * dot_rmsprop_step -- one RMSProp update of the sigma and SH planes in place
 *  (the optimiser of Sec. 3.3): v = alpha v + (1 - alpha) g^2,
 *  theta -= lr g / (sqrt(v) + eps).  grad_*: DEVICE float, dense layouts as in
 *  dot_render_backward; v_*: DEVICE float square averages of the same shapes,
 *  zero-initialised by the caller.  FP32 storage only (DOT_EUNSUPPORTED
 *  otherwise); DOT_EINVAL for alpha outside [0, 1) or eps not positive.
 */
int dot_rmsprop_step(dot_tree_t tree, const float *grad_sigma, const float *grad_sh, float *v_sigma,
                     float *v_sh, const dot_rmsprop_params *params, void *stream);

/*
 * dot_render_backward_rmsprop -- dot_render_backward followed by one
 *  dot_rmsprop_step, fused: each leaf's bucket sums (its gradient) feed the
 *  update directly, so the dense gradient arrays are neither zeroed, written
 *  nor read back.  Same arithmetic as dot_render_backward into zeroed arrays
 *  followed by dot_rmsprop_step; every leaf is updated (a leaf no ray reached
 *  has g = 0: its square average decays, its values stay).  Arguments as in
 *  those two calls.  When the bucket scratch cannot be used the call falls
 *  back to dense gradients from the tree's allocator (DOT_ENOMEM if that
 *  fails too).  FP32 storage only (DOT_EUNSUPPORTED otherwise).
 */
int dot_render_backward_rmsprop(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts,
                                const float *rgb_fwd, const int32_t *nseg, const float *grad_rgb, float *v_sigma,
                                float *v_sh, const dot_rmsprop_params *params, const uint32_t *leaf_count,
                                const void *records, size_t records_bytes, void *stream);

/*
 * dot_render_backward_adam -- dot_render_backward followed by one
 *  dot_adam_step, fused in the same way as dot_render_backward_rmsprop: each
 *  leaf's bucket sums feed the update directly and no dense gradient array
 *  exists.  Same arithmetic as dot_render_backward into zeroed arrays followed
 *  by dot_adam_step; every leaf is updated (a leaf no ray reached has g = 0:
 *  both moments decay and its values still move by the decayed first moment).
 *  Arguments and errors as in those two calls; the same dense fallback as
 *  dot_render_backward_rmsprop.  FP32 storage only (DOT_EUNSUPPORTED
 *  otherwise).
 */
int dot_render_backward_adam(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts,
                             const float *rgb_fwd, const int32_t *nseg, const float *grad_rgb, float *m_sigma,
                             float *v_sigma, float *m_sh, float *v_sh, const dot_adam_params *params,
                             const uint32_t *leaf_count, const void *records, size_t records_bytes, void *stream);

/*
 * dot_sigma_signal -- the density as the training signal (the paper's Pr_sigma
 *  ablation, Sec. 3.1 and Tab. 3): signal_out[l] = max(sigma_l, 0) decoded to
 *  FP32.  signal_out: DEVICE float [n_leaves].
 */
int dot_sigma_signal(dot_tree_t tree, float *signal_out, void *stream);

/*
 * dot_pixel_batch -- a batch of training rays for one optimisation step
 *  (Alg. 1: the rays are permuted each epoch and consumed batch by batch).
 *  ray_ids: DEVICE int64 [n] flat pixel ids cam * H * W + v * W + u over
 *  n_cams cameras of width x height (a slice of the epoch's permutation).
 *  Writes the same rays as a DOT_RAYS_PIXELS list, cam_idx_out / pix_idx_out
 *  (DEVICE int32 [n]), grouped by screen tile -- square tiles sized to hold
 *  about 16 of the batch's rays, in camera-then-row-major tile order; order
 *  inside a tile unspecified -- so that a wave traces neighbouring pixels.
 *  ray_ids_out (DEVICE int64 [n] or NULL) receives the ids in the new order,
 *  for use as the target rows of dot_mse_loss.  The batch's content is
 *  unchanged (the loss is a mean and the gradient a sum over it).
 *  workspace: DEVICE, at least dot_pixel_batch_workspace(n, width, height,
 *  n_cams) bytes, caller-owned, clobbered.  An id outside [0, n_cams*H*W) is a
 *  contract violation; it is replaced by 0 so no access leaves the arrays.
 *  Errors: DOT_EINVAL on n < 0, non-positive sizes, more than 2^31 pixels per
 *  image, NULL buffers with n > 0, or a workspace that is too small.
 */
size_t dot_pixel_batch_workspace(int64_t n_rays, int32_t width, int32_t height, int32_t n_cams);
int dot_pixel_batch(const int64_t *ray_ids, int64_t n_rays, int32_t width, int32_t height, int32_t n_cams,
                    int32_t *cam_idx_out, int32_t *pix_idx_out, int64_t *ray_ids_out, void *workspace,
                    size_t workspace_bytes, void *stream);

/*
 * dot_pixel_batch_noalloc -- dot_pixel_batch without a workspace argument, for
 *  callers that cannot allocate device memory (code under HIP graph capture,
 *  serving or training loops that forbid allocation).  Same arguments, outputs
 *  and ordering contract as dot_pixel_batch; the scratch is a device array of
 *  DOT_PIXEL_BATCH_SCRATCH_BYTES that the library holds on every GPU it runs
 *  on until the process ends (found once per device, with that device
 *  current).  The call allocates nothing.  All calls on one GPU share that
 *  array, which keeps the last call's contents (the kernels clear what must
 *  start at zero): calls that overlap on one GPU (on different streams, or
 *  from different threads) race and give wrong orders.
 *  Errors: as dot_pixel_batch, and DOT_EINVAL (before any device work) when
 *  the batch needs more than DOT_PIXEL_BATCH_SCRATCH_BYTES of scratch, i.e.
 *  when dot_pixel_batch_workspace(n, width, height, n_cams) exceeds it: about
 *  4 bytes per ray plus 8 per screen tile, so batches of up to 2^21 rays fit
 *  for any image set with fewer than 400,000 tiles, and about 3.5M rays of
 *  100 views at 800x800.
 */
#define DOT_PIXEL_BATCH_SCRATCH_BYTES (16u << 20)
int dot_pixel_batch_noalloc(const int64_t *ray_ids, int64_t n_rays, int32_t width, int32_t height, int32_t n_cams,
                            int32_t *cam_idx_out, int32_t *pix_idx_out, int64_t *ray_ids_out, void *stream);

/*
 * dot_mse_loss -- the photometric loss of a training step (Sec. 3 and Alg. 1:
 *  the prediction of a permuted ray batch against its ground-truth pixels)
 *  and its gradient with respect to the prediction:
 *      loss        = 1/(3n) sum_r sum_ch (pred[r][ch] - target[idx_r][ch])^2
 *      grad_rgb[r] = 2 (pred[r] - target[idx_r]) / (3n)
 *  pred: DEVICE float [n][3]; target: DEVICE float [*][3]; target_idx: DEVICE
 *  int64 [n] (row of `target` that ray r is compared with, which the caller
 *  guarantees to be in range) or NULL (row r); grad_rgb_out: DEVICE float
 *  [n][3] or NULL; loss_out: DEVICE double [1] or NULL, overwritten.  Residuals
 *  and the sum are formed in FP64 (the gradient is rounded once to FP32; the
 *  summation order depends on scheduling).  n_rays = 0 writes a zero loss.
 *  Errors: DOT_EINVAL on n_rays < 0 or a NULL pred/target with n_rays > 0.
 */
int dot_mse_loss(const float *pred, const float *target, const int64_t *target_idx, int64_t n_rays,
                 float *grad_rgb_out, double *loss_out, void *stream);

/*
 * dot_mse_grad -- the gradient of dot_mse_loss times a factor that lives on
 *  the device (the upstream gradient of the loss when the loss is itself
 *  differentiated by a caller's chain rule, Sec. 3):
 *      grad_rgb[r] = s * 2 (pred[r] - target[idx_r]) / (3n),   s = *scale
 *  scale: DEVICE double [1], or NULL for s = 1 (then the gradient equals
 *  dot_mse_loss's bit for bit); the product 2s/(3n) and the residual are
 *  formed in FP64 and rounded once.  Other arguments as dot_mse_loss;
 *  grad_rgb_out is required when n_rays > 0.
 *  Errors: DOT_EINVAL on n_rays < 0, or a NULL pred/target/grad_rgb_out with
 *  n_rays > 0.
 */
int dot_mse_grad(const float *pred, const float *target, const int64_t *target_idx, int64_t n_rays,
                 const double *scale, float *grad_rgb_out, void *stream);

/*
 * dot_quantize_sh -- compress the tree's SH coefficients into a palette (the
 *  compressed octrees of Sec. 4.1, quantised with Heckbert's median cut).
 *  Each leaf's SH row (3K values as stored) is a point; `bits` rounds each cut
 *  every box at the median of its widest dimension (largest max - min, ties:
 *  lowest dimension; members ordered by value then leaf index, -0.0 = +0.0;
 *  the lower n/2 go to box 2b, the rest to 2b + 1), giving 2^bits boxes (some
 *  empty when there are few leaves).  A palette row is the FP64 mean of its
 *  box rounded once to FP16 (zero for an empty box); each leaf keeps the
 *  uint16 index of its box.  The tree becomes DOT_PAL16 in place (sigma
 *  rounded to FP16).  Rendering, serving, the signal calls and dot_export
 *  accept it; dot_render_backward, the optimiser steps and dot_refine return
 *  DOT_EUNSUPPORTED.  Needs scratch of about 2 N (3K + 4) * 4 bytes from the
 *  tree's allocator; synchronises `stream`.
 *  Errors: DOT_EINVAL on bits outside 1..16 or an already compressed tree;
 *  DOT_ENOMEM when the scratch cannot be allocated.
 */
int dot_quantize_sh(dot_tree_t tree, int32_t bits, void *stream);

/*
 * dot_export -- copy the tree back to host memory in canonical form:
 *  child [n_internal][8], sigma [L] and sh [L][3][K] decoded to FP32,
 *  leaf_depth [L].  Any pointer may be NULL.  Synchronous.
 */
int dot_export(dot_tree_t tree, int32_t *child, float *sigma, float *sh, uint8_t *leaf_depth,
               void *stream);

/*
 * dot_render_stats -- work counters of one forward pass over `rays` (no colour
 *  output): counts[0] rays, [1] segments composited (delta > 0), [2] segments
 *  whose SH coefficients were fetched (sigma^ delta > 0), [3] child-array
 *  and neighbour-link reads (4 B each) during traversal.  Synchronous.  Used
 *  to turn kernel time into algorithmic bytes per second.
 */
int dot_render_stats(dot_tree_t tree, const dot_rays *rays, const dot_render_opts *opts,
                     int64_t counts[4], void *stream);

/*
 * Batched rendering for serving: many render requests, over several resident
 * trees, in one launch.  A job renders the 8x8 pixel tiles
 * [tile_begin, tile_begin + tile_count) of one request's image (tiles are
 * numbered row-major over ceil(width/8) x ceil(height/8)); a large request can
 * therefore be split over several launches and mixed with others.  The image
 * of each pixel is exactly what dot_render computes for the same camera and
 * options (Eq. 1-2), independent of the rest of the batch.
 */
typedef struct {
    dot_tree_t tree;         /* resident tree */
    const dot_camera *cam;   /* DEVICE pointer to one camera record */
    float *rgb_out;          /* DEVICE float [height][width][3] */
    int32_t width, height;
    int64_t tile_begin, tile_count;
    float bg[3];
    float t_stop;
} dot_render_job;

/* dot_render_jobs_workspace -- bytes of device workspace a launch of n_jobs needs. */
size_t dot_render_jobs_workspace(int32_t n_jobs);

/*
 * dot_render_jobs -- one persistent launch over all tiles of `jobs` (host
 *  array, read during the call) per leaf storage type present among them
 *  (usually one), each with the registers of its own type.  Tiles are handed
 *  out in 8 contiguous chunks, one per XCD, with stealing between chunks.
 *  `workspace` is a DEVICE buffer of at least
 *  dot_render_jobs_workspace(n_jobs) bytes owned by the caller; the call
 *  writes the job table into it on `stream`, so it may be reused by the next
 *  call on the same stream, but not concurrently on another stream.
 *  Errors: DOT_EINVAL for a NULL tree/camera/output, a tile range outside the
 *  image, or a small workspace.
 */
int dot_render_jobs(const dot_render_job *jobs, int32_t n_jobs, void *workspace, size_t workspace_bytes,
                    void *stream);

/*
 * Persistent serving queue: ONE launch that stays on the device and renders
 * the jobs the host appends while it runs, so a request that arrives while
 * others are on the GPU is admitted without waiting for a launch to end, and
 * the tiles of all admitted requests are rendered by the same resident waves.
 * The host writes each job into a ring in pinned, host-coherent memory and
 * publishes it with a counter; one wave of the launch copies published jobs
 * into device memory and schedules their tiles onto one tile ring per XCD, a
 * share at a time beside the other jobs in flight (so a small request is not
 * queued behind every tile of a large one); the wave that renders a job's
 * last tile writes the job's completion word back to host memory, after the
 * job's pixels are visible to other device work (a copy on another stream may
 * read the image as soon as dot_serve_done reports it, while the launch runs).
 * Every pixel is computed by the same per-ray code
 * as dot_render (Eq. 1-2), so a job's image does not depend on what else is
 * queued.  One queue serves trees of one storage type (the launch carries that
 * type's registers), at most `max_jobs` jobs in flight and 2^19 tiles of
 * unfinished jobs; images of at most 2^20 tiles.  The launch holds all but one
 * workgroup slot per compute unit until it is closed: other device work can
 * run beside it in the slot left free, but work that needs the whole GPU, or
 * a host wait on such work, must not be issued while a queue is open.
 */
typedef struct dot_serve_queue *dot_serve_t;

typedef struct {
    dot_tree_t tree;         /* resident tree of the queue's storage type */
    dot_camera cam;          /* by value */
    float *rgb_out;          /* DEVICE float [height][width][3]; written when the job completes */
    int32_t width, height;
    int64_t tile_begin, tile_count;   /* 8x8 tiles [begin, begin + count) of the image, count >= 1 */
    float bg[3];
    float t_stop;
} dot_serve_job;

/*
 * dot_serve_open -- allocate a queue (pinned host ring, device state) and
 *  launch its kernel on `stream`, which it occupies until dot_serve_close.
 *  storage: DOT_F32 / DOT_F16 / DOT_BF16 / DOT_PAL16; max_jobs in 1..4096.
 *  max_seconds > 0: the launch ends by itself after that long (jobs still
 *  queued are then never completed and dot_serve_done reports DOT_EHIP), so it
 *  can never outlive a host that stopped serving.
 *  Errors: DOT_EINVAL on bad arguments; DOT_ENOMEM / DOT_EHIP from the runtime.
 */
int dot_serve_open(int32_t storage, int32_t max_jobs, double max_seconds, void *stream, dot_serve_t *out);

/*
 * dot_serve_push -- append one job (host call, returns at once); *ticket
 *  receives its number for dot_serve_done.  The camera is copied; the tree and
 *  rgb_out must stay valid until the job completes.  Not thread-safe per queue.
 *  Errors: DOT_EINVAL for a NULL tree/output, a tree of another storage type,
 *  a bad size, tile range or t_stop; DOT_EBUSY when max_jobs jobs or 2^19
 *  tiles are unfinished (nothing is queued; retry later); DOT_EHIP after the
 *  launch ended (closed, or past max_seconds).
 */
int dot_serve_push(dot_serve_t q, const dot_serve_job *job, int64_t *ticket);

/*
 * dot_serve_done -- 1 when job `ticket` has been rendered (its rgb_out is
 *  complete and visible to device work issued after this call, on any stream,
 *  also while the launch keeps running), 0 while it is pending.
 *  Errors: DOT_EINVAL for an unknown ticket; DOT_EHIP when the launch ended
 *  before the job completed.
 */
int dot_serve_done(dot_serve_t q, int64_t ticket);

/*
 * dot_serve_close -- tell the launch that no job will follow, wait until it
 *  has rendered every published job and ended, then free the queue.  The
 *  launch ends by its own clock within 9/8 of max_seconds in any case; the
 *  call waits at most 5/4 of max_seconds plus 10 s.
 *  Errors: DOT_EHIP if the launch has not ended by then (the queue is then
 *  left allocated).
 */
int dot_serve_close(dot_serve_t q);

/*
 * dot_stream_read -- support kernel, not part of the method: reads `bytes`
 *  (rounded down to 16) of the DEVICE buffer `buf` once with 16-byte loads,
 *  to measure the achievable HBM read bandwidth that the renderer's roofline is
 *  set against.  sink: DEVICE float, receives a value only to keep the loads
 *  live.  Errors: DOT_EINVAL on a NULL or unaligned buffer.
 */
int dot_stream_read(const void *buf, size_t bytes, float *sink, void *stream);

/*
 * dot_gather_rows -- support kernel, not part of the method: reads about
 *  `reads` rows of 192 bytes (the FP32 SH row of a leaf), each lane a whole
 *  row per step, at positions spread over the first n_rows rows of the DEVICE
 *  buffer `buf` by a 64-bit mixing hash; the achievable rate of the
 *  renderer's leaf-fetch pattern without its dependences (the ceiling beside
 *  dot_stream_read's).  The number of rows read is rounded to a multiple of
 *  the launch's threads (at least one per thread); the caller times the call.
 *  buf: DEVICE, at least n_rows * 192 bytes, 16-byte aligned; n_rows a power
 *  of two; sink: DEVICE float, receives a value only to keep the loads live.
 *  Errors: DOT_EINVAL on a NULL or unaligned buffer or n_rows not a power of
 *  two.
 */
int dot_gather_rows(const void *buf, int64_t n_rows, int64_t reads, float *sink, void *stream);

/*
 * dot_atomic_count -- support kernel, not part of the method: n device-wide
 *  32-bit atomic increments, the i-th to counter (64-bit mix of i) mod
 *  n_counters of the DEVICE array `counters` (added to, not cleared); with
 *  `returning` nonzero each increment's returned value is used.  The pattern
 *  of the training forward's per-leaf segment counts (and its slot
 *  reservations) without the rest of its work: the rate it cannot exceed.  The
 *  caller times the call; afterwards the counters have grown by n in total.
 *  Errors: DOT_EINVAL for n < 0, or n > 0 with NULL counters or n_counters 0.
 */
int dot_atomic_count(uint32_t *counters, uint32_t n_counters, int64_t n, int returning, void *stream);

/* dot_last_error -- message of the last failure on this thread ("" if none). */
const char *dot_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DOT_H_ */
