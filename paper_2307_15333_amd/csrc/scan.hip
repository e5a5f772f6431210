// Exclusive prefix scan of uint32 arrays: per-tile sums, a single-workgroup
// scan of the tile sums, then a per-tile rescan with the tile's offset; arrays
// of up to 16 tiles are scanned by one workgroup in one launch.
#include <hip/hip_runtime.h>

#include "dot_internal.h"

namespace dot {

namespace {
constexpr int TPB = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = TPB * SCAN_ITEMS;

template <int NT = TPB>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t& total) {
    __shared__ uint32_t wsum[NT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t base = 0;
    total = 0;
#pragma unroll
    for (int j = 0; j < NT / 64; ++j) {
        if (j < w) base += wsum[j];
        total += wsum[j];
    }
    __syncthreads();
    return base + x - v;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + (int64_t)j * TPB + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t total;
    block_exclusive_scan(acc, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// single block: exclusive scan of the block sums in place; total into *tot
__global__ void k_scan_bsums(uint32_t* __restrict__ bsum, int64_t nb, uint32_t* __restrict__ tot) {
    const int64_t per = (nb + TPB - 1) / TPB;
    const int64_t b0 = threadIdx.x * per;
    uint32_t acc = 0;
    for (int64_t i = b0; i < b0 + per && i < nb; ++i) acc += bsum[i];
    uint32_t total;
    uint32_t off = block_exclusive_scan(acc, total);
    for (int64_t i = b0; i < b0 + per && i < nb; ++i) {
        uint32_t v = bsum[i];
        bsum[i] = off;
        off += v;
    }
    if (threadIdx.x == 0) *tot = total;
}

// A thread's SCAN_ITEMS consecutive elements from base: four 16-byte loads when
// VEC (both arrays 16-byte aligned) and the run lies inside the array, else
// element by element; store_run writes the exclusive prefix from `off`.
template <bool VEC>
__device__ __forceinline__ uint32_t load_run(const uint32_t* __restrict__ in, int64_t base, int64_t n,
                                             uint32_t (&v)[SCAN_ITEMS]) {
    if (VEC && base + SCAN_ITEMS <= n) {
        const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS / 4; ++q) {
            const uint4 x = p[q];
            v[4 * q] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) v[j] = base + j < n ? in[base + j] : 0u;
    }
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) acc += v[j];
    return acc;
}

template <bool VEC>
__device__ __forceinline__ void store_run(uint32_t* __restrict__ out, int64_t base, int64_t n,
                                          const uint32_t (&v)[SCAN_ITEMS], uint32_t off) {
    if (VEC && base + SCAN_ITEMS <= n) {
        uint4* p = reinterpret_cast<uint4*>(out + base);
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS / 4; ++q) {
            uint4 x;
            x.x = off;
            off += v[4 * q];
            x.y = off;
            off += v[4 * q + 1];
            x.z = off;
            off += v[4 * q + 2];
            x.w = off;
            off += v[4 * q + 3];
            p[q] = x;
        }
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            if (base + j < n) out[base + j] = off;
            off += v[j];
        }
    }
}

// a thread's SCAN_ITEMS consecutive values, stored as they are
template <bool VEC>
__device__ __forceinline__ void store_vals(uint32_t* __restrict__ out, int64_t base, int64_t n,
                                           const uint32_t (&v)[SCAN_ITEMS]) {
    if (VEC && base + SCAN_ITEMS <= n) {
        uint4* p = reinterpret_cast<uint4*>(out + base);
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS / 4; ++q) p[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j)
            if (base + j < n) out[base + j] = v[j];
    }
}

template <bool VEC>
__global__ void k_scan_apply(const uint32_t* __restrict__ in, int64_t n, const uint32_t* __restrict__ bsum,
                             uint32_t* __restrict__ out) {
    // each thread owns SCAN_ITEMS consecutive elements of the tile
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    const uint32_t acc = load_run<VEC>(in, base, n, v);
    uint32_t total;
    const uint32_t off = block_exclusive_scan(acc, total) + bsum[blockIdx.x];
    store_run<VEC>(out, base, n, v, off);
}

// small arrays: one workgroup of 1024 threads walks tiles of 16K elements in
// order, carrying the running total (one launch instead of three; an array of
// up to 16K elements is one tile, so one load round trip)
constexpr int SINGLE_TPB = 1024;
constexpr int64_t SINGLE_TILE = (int64_t)SINGLE_TPB * SCAN_ITEMS;
constexpr int64_t SCAN_SINGLE_MAX = 16 * SCAN_TILE;

template <bool VEC>
__global__ __launch_bounds__(SINGLE_TPB) void k_scan_single(const uint32_t* __restrict__ in, int64_t n,
                                                            uint32_t* __restrict__ out, uint32_t* __restrict__ tot) {
    uint32_t carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += SINGLE_TILE) {
        const int64_t base = t0 + (int64_t)threadIdx.x * SCAN_ITEMS;
        uint32_t v[SCAN_ITEMS];
        const uint32_t acc = load_run<VEC>(in, base, n, v);
        uint32_t total;
        const uint32_t off = block_exclusive_scan<SINGLE_TPB>(acc, total) + carry;
        store_run<VEC>(out, base, n, v, off);
        carry += total;
    }
    if (threadIdx.x == 0) *tot = carry;
}

// the same over a + b (a bucket's two count regions), also writing the sum
// to c and zeroing z (the bucket cursors); the first thread copies *w_src to
// *w_dst (a word the host may read back with the total)
template <bool VEC>
__global__ __launch_bounds__(SINGLE_TPB) void k_scan_single_sum2(const uint32_t* __restrict__ a,
                                                                 const uint32_t* __restrict__ b, int64_t n,
                                                                 uint32_t* __restrict__ c, uint32_t* __restrict__ z,
                                                                 uint32_t* __restrict__ out, uint32_t* __restrict__ tot,
                                                                 const uint32_t* __restrict__ w_src,
                                                                 uint32_t* __restrict__ w_dst) {
    if (w_src && threadIdx.x == 0) *w_dst = *w_src;
    uint32_t carry = 0;
    const uint32_t zero[SCAN_ITEMS] = {};
    for (int64_t t0 = 0; t0 < n; t0 += SINGLE_TILE) {
        const int64_t base = t0 + (int64_t)threadIdx.x * SCAN_ITEMS;
        uint32_t v[SCAN_ITEMS], w[SCAN_ITEMS];
        const uint32_t acc = load_run<VEC>(a, base, n, v) + load_run<VEC>(b, base, n, w);
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) v[j] += w[j];
        store_vals<VEC>(c, base, n, v);
        store_vals<VEC>(z, base, n, zero);
        uint32_t total;
        const uint32_t off = block_exclusive_scan<SINGLE_TPB>(acc, total) + carry;
        store_run<VEC>(out, base, n, v, off);
        carry += total;
    }
    if (threadIdx.x == 0) *tot = carry;
}

}  // namespace

int64_t scan_scratch_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

bool scan_u32_sum2(const uint32_t* a, const uint32_t* b, uint32_t* c, uint32_t* z, uint32_t* out, int64_t n,
                   uint32_t* tot, const uint32_t* w_src, uint32_t* w_dst, hipStream_t s, hipError_t* err) {
    if (n <= 0 || n > SCAN_SINGLE_MAX) return false;
    const bool vec = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c) |
                       reinterpret_cast<uintptr_t>(z) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (vec)
        hipLaunchKernelGGL(k_scan_single_sum2<true>, dim3(1), dim3(SINGLE_TPB), 0, s, a, b, n, c, z, out, tot, w_src, w_dst);
    else
        hipLaunchKernelGGL(k_scan_single_sum2<false>, dim3(1), dim3(SINGLE_TPB), 0, s, a, b, n, c, z, out, tot, w_src, w_dst);
    *err = hipGetLastError();
    return true;
}

hipError_t scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* bsum, uint32_t* tot, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (n <= SCAN_SINGLE_MAX) {
        if (vec)
            hipLaunchKernelGGL(k_scan_single<true>, dim3(1), dim3(SINGLE_TPB), 0, s, in, n, out, tot);
        else
            hipLaunchKernelGGL(k_scan_single<false>, dim3(1), dim3(SINGLE_TPB), 0, s, in, n, out, tot);
        return hipGetLastError();
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(TPB), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(TPB), 0, s, bsum, nb, tot);
    if (vec)
        hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)nb), dim3(TPB), 0, s, in, n, bsum, out);
    else
        hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)nb), dim3(TPB), 0, s, in, n, bsum, out);
    return hipGetLastError();
}

}  // namespace dot
