// Training-batch preparation: a batch of training rays given as flat pixel ids
// (cam * H * W + v * W + u, a slice of the epoch's random permutation) becomes
// a (camera, pixel) ray list grouped by screen tile, so that the 64 lanes of a
// wave trace neighbouring pixels of one camera and share the leaves they
// fetch.  A counting sort: per-tile counts, an exclusive scan, a scatter.
// The batch's content is unchanged; only its order is (the loss is a mean and
// the gradient a sum over the batch).
#include <hip/hip_runtime.h>

#include <mutex>

#include "dot_internal.h"

namespace dot {

namespace {

struct PixelGeo {
    int32_t W, H, shift, tw;
    int64_t tpv;      // tiles per camera
    int64_t total;    // n_cams * W * H
    int64_t bins;     // n_cams * tpv
};

// tile edge 2^shift: the smallest (8 to 128 pixels) whose tile holds about 16
// of the batch's rays, so a wave takes the rays of a few neighbouring tiles.
// (Measured on 2^20 random rays of 100 800x800 views: a step of the training
// loop is 4% faster than with about 64 rays per tile, where a wave's rays
// spread over a tile twice as wide; numbering the tiles in Morton order
// instead of row-major gave nothing more.)
constexpr double RAYS_PER_TILE = 16.0;

PixelGeo make_geo(int64_t n, int32_t W, int32_t H, int32_t n_cams) {
    PixelGeo g;
    g.W = W;
    g.H = H;
    g.total = (int64_t)n_cams * W * H;
    const double density = g.total > 0 ? (double)n / (double)g.total : 1.0;
    int shift = 3;
    while (shift < 7 && (double)(1 << (2 * shift)) * density < RAYS_PER_TILE) ++shift;
    g.shift = shift;
    g.tw = (W + (1 << shift) - 1) >> shift;
    g.tpv = (int64_t)g.tw * ((H + (1 << shift) - 1) >> shift);
    g.bins = (int64_t)n_cams * g.tpv;
    return g;
}

__device__ __forceinline__ int64_t tile_bin(int64_t& id, const PixelGeo& g, int32_t& cam, int32_t& pix) {
    if (id < 0 || id >= g.total) id = 0;   // outside the image set: replaced by ray 0 (documented)
    const int64_t hw = (int64_t)g.W * g.H;
    cam = (int32_t)(id / hw);
    pix = (int32_t)(id - (int64_t)cam * hw);
    const int v = pix / g.W, u = pix - v * g.W;
    return (int64_t)cam * g.tpv + (int64_t)(v >> g.shift) * g.tw + (u >> g.shift);
}

__global__ void k_pb_zero(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Many bins: one global atomic per ray, whose return value is the ray's rank
// in its bin, so the scatter needs none (offset[bin] + rank).
__global__ void k_pb_count(const int64_t* __restrict__ ids, int64_t n, PixelGeo g, uint32_t* __restrict__ count,
                           uint32_t* __restrict__ rank) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        int64_t id = ids[r];
        int32_t cam, pix;
        rank[r] = atomicAdd(&count[tile_bin(id, g, cam, pix)], 1u);
    }
}

__global__ void k_pb_scatter(const int64_t* __restrict__ ids, int64_t n, PixelGeo g, const uint32_t* __restrict__ offset,
                             const uint32_t* __restrict__ rank, int32_t* __restrict__ cam_out,
                             int32_t* __restrict__ pix_out, int64_t* __restrict__ id_out) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        int64_t id = ids[r];
        int32_t cam, pix;
        const int64_t b = tile_bin(id, g, cam, pix);
        const uint32_t pos = offset[b] + rank[r];
        cam_out[pos] = cam;
        pix_out[pos] = pix;
        if (id_out) id_out[pos] = id;
    }
}

// Few bins: every workgroup counts (and ranks) its chunk of rays in LDS, so a
// bin takes one global atomic per workgroup instead of one per ray.
constexpr int LDS_BINS = 4096;
constexpr int ITEMS = 4;                // rays per thread
constexpr int CHUNK = 256 * ITEMS;      // rays per workgroup

__global__ __launch_bounds__(256) void k_pb_count_lds(const int64_t* __restrict__ ids, int64_t n, PixelGeo g,
                                                      uint32_t* __restrict__ count) {
    __shared__ uint32_t h[LDS_BINS];
    for (int i = threadIdx.x; i < g.bins; i += 256) h[i] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * CHUNK;
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * 256 + threadIdx.x;
        if (r < n) {
            int64_t id = ids[r];
            int32_t cam, pix;
            atomicAdd(&h[tile_bin(id, g, cam, pix)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < g.bins; i += 256)
        if (h[i]) atomicAdd(&count[i], h[i]);
}

// cursor holds each bin's exclusive offset; a workgroup reserves one range per
// bin for its rays, then places each ray at its LDS rank within that range
__global__ __launch_bounds__(256) void k_pb_scatter_lds(const int64_t* __restrict__ ids, int64_t n, PixelGeo g,
                                                        uint32_t* __restrict__ cursor, int32_t* __restrict__ cam_out,
                                                        int32_t* __restrict__ pix_out, int64_t* __restrict__ id_out) {
    __shared__ uint32_t h[LDS_BINS];
    __shared__ uint32_t b0[LDS_BINS];
    for (int i = threadIdx.x; i < g.bins; i += 256) h[i] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * CHUNK;
    uint32_t bin[ITEMS], rank[ITEMS];
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * 256 + threadIdx.x;
        if (r < n) {
            int64_t id = ids[r];
            int32_t cam, pix;
            bin[j] = (uint32_t)tile_bin(id, g, cam, pix);
            rank[j] = atomicAdd(&h[bin[j]], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < g.bins; i += 256) b0[i] = h[i] ? atomicAdd(&cursor[i], h[i]) : 0u;
    __syncthreads();
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * 256 + threadIdx.x;
        if (r < n) {
            int64_t id = ids[r];
            int32_t cam, pix;
            (void)tile_bin(id, g, cam, pix);
            const uint32_t pos = b0[bin[j]] + rank[j];
            cam_out[pos] = cam;
            pix_out[pos] = pix;
            if (id_out) id_out[pos] = id;
        }
    }
}

unsigned grid_of(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

size_t pixel_batch_workspace_bytes(int64_t n, int32_t W, int32_t H, int32_t n_cams) {
    const PixelGeo g = make_geo(n, W, H, n_cams);
    const int64_t ranks = g.bins <= LDS_BINS ? 0 : n;    // the many-bin path keeps each ray's rank
    return sizeof(uint32_t) * (size_t)(2 * g.bins + scan_scratch_elems(g.bins) + 1 + ranks);
}

hipError_t launch_pixel_batch(const int64_t* ids, int64_t n, int32_t W, int32_t H, int32_t n_cams, int32_t* cam_out,
                              int32_t* pix_out, int64_t* id_out, void* ws, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const PixelGeo g = make_geo(n, W, H, n_cams);
    uint32_t* count = static_cast<uint32_t*>(ws);
    uint32_t* cursor = count + g.bins;
    uint32_t* bsum = cursor + g.bins;
    uint32_t* tot = bsum + scan_scratch_elems(g.bins);
    uint32_t* rank = tot + 1;
    const bool lds = g.bins <= LDS_BINS;
    const unsigned gl = (unsigned)((n + CHUNK - 1) / CHUNK);
    hipLaunchKernelGGL(k_pb_zero, dim3(grid_of(g.bins)), dim3(256), 0, s, count, g.bins);
    if (lds)
        hipLaunchKernelGGL(k_pb_count_lds, dim3(gl), dim3(256), 0, s, ids, n, g, count);
    else
        hipLaunchKernelGGL(k_pb_count, dim3(grid_of(n)), dim3(256), 0, s, ids, n, g, count, rank);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = scan_u32(count, cursor, g.bins, bsum, tot, s);
    if (e != hipSuccess) return e;
    if (lds)
        hipLaunchKernelGGL(k_pb_scatter_lds, dim3(gl), dim3(256), 0, s, ids, n, g, cursor, cam_out, pix_out, id_out);
    else
        hipLaunchKernelGGL(k_pb_scatter, dim3(grid_of(n)), dim3(256), 0, s, ids, n, g, cursor, rank, cam_out, pix_out,
                           id_out);
    return hipGetLastError();
}

// Scratch of the no-allocation entry point: one array per GPU, held until the
// process ends.  In host code `scratch` is only a stand-in for the symbol; the
// kernels receive the device address hipGetSymbolAddress gives for the current
// device, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[DOT_PIXEL_BATCH_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t pixel_batch_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace dot
