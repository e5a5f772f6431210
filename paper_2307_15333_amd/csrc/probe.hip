// Device probes: the achievable HBM read bandwidth (streaming and random
// rows), the ceilings beside the 8 TB/s specification in the renderer's
// roofline, and the device-wide atomic rate that bounds the training
// forward's per-leaf counting.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dot_internal.h"

namespace dot {

namespace {

// every workgroup reduces a strided share of the buffer with 16-byte
// non-temporal loads (four independent loads in flight per thread) and the
// partial of each wave is compared with a fixed pattern that adds to *sink
// (practically never equal), so the loads cannot be dropped.
// Non-temporal loads, four in flight and two workgroups of 256 per CU read
// fastest in a sweep of load kind x loads in flight (2..16) x workgroups per
// CU (2..64) over a 4 GiB buffer.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t fold(const v4u* p) {
    const v4u v = __builtin_nontemporal_load(p);
    return v.x ^ v.y ^ v.z ^ v.w;
}

__global__ __launch_bounds__(256) void k_stream_read(const v4u* __restrict__ p, int64_t n16, float* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < n16; i += 4 * stride)
        acc ^= fold(p + i) ^ fold(p + i + stride) ^ fold(p + i + 2 * stride) ^ fold(p + i + 3 * stride);
    for (; i < n16; i += stride) acc ^= fold(p + i);
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0 && acc == 0x7fc00001u) atomicAdd(sink, 1.f);   // practically never taken
}

// Gather probe: every lane reads whole 192-byte rows (twelve 16-byte loads,
// the FP32 SH row of a leaf) at positions spread over the buffer by a 64-bit
// mixing function (the splitmix64 finalizer of Steele, Lea and Flood), the
// access pattern of the renderer's leaf fetches without its dependences.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_gather_rows(const v4u* __restrict__ p, uint64_t row_mask, int64_t trips,
                                                    float* __restrict__ sink) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int64_t t = 0; t < trips; ++t) {
        const uint64_t r = mix64(tid * (uint64_t)trips + (uint64_t)t) & row_mask;
        v4u v[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) v[q] = p[r * 12 + q];
#pragma unroll
        for (int q = 0; q < 12; ++q) acc ^= v[q].x ^ v[q].y ^ v[q].z ^ v[q].w;
    }
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0 && acc == 0x7fc00001u) atomicAdd(sink, 1.f);   // practically never taken
}

// Atomic probe: n device-wide 32-bit increments, the i-th to counter
// mix64(i) mod K, the access pattern of the training forward's per-leaf
// segment counts without its other work; with `ret` the returned values are
// folded into a register (as the forward's slot reservations use theirs).
__global__ __launch_bounds__(256) void k_atomic_count(uint32_t* __restrict__ c, uint32_t K, int64_t n, int ret) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t k = (uint32_t)(mix64((uint64_t)i) % K);
        if (ret)
            acc += atomicAdd(&c[k], 1u);
        else
            atomicAdd(&c[k], 1u);
    }
    if (ret && acc == 0x7fc00001u) atomicAdd(&c[0], 0u);   // keeps the returned values live; adds nothing
}

}  // namespace

hipError_t launch_atomic_count(uint32_t* counters, uint32_t n_counters, int64_t n, bool returning, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 256;
    }
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)cus * 8);
    hipLaunchKernelGGL(k_atomic_count, dim3((unsigned)blocks), dim3(256), 0, s, counters, n_counters, n,
                       returning ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const void* buf, int64_t n_rows_pow2, int64_t reads, float* sink, hipStream_t s) {
    if (n_rows_pow2 <= 0 || reads <= 0) return hipSuccess;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 256;
    }
    // four workgroups of 256 per CU (the rate is flat from 2 to 16), each
    // thread taking reads / threads rows in turn
    const int64_t threads = (int64_t)cus * 4 * 256;
    const int64_t trips = std::max<int64_t>(1, reads / threads);
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)(cus * 4)), dim3(256), 0, s, static_cast<const v4u*>(buf),
                       (uint64_t)(n_rows_pow2 - 1), trips, sink);
    return hipGetLastError();
}

hipError_t launch_stream_read(const void* buf, size_t bytes, float* sink, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 256;
    }
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, (int64_t)cus * 2);
    hipLaunchKernelGGL(k_stream_read, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const v4u*>(buf), n16, sink);
    return hipGetLastError();
}

}  // namespace dot
