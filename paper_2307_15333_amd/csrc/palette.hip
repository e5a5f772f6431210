// Median-cut palette of the SH coefficients (the compressed octrees of
// Sec. 4.1, Heckbert's median cut).  Every leaf's SH row (3K values) is a point;
// in each of `bits` rounds every box is cut at the median of its widest
// dimension (ties: lowest dimension; members ordered by value, then leaf
// index; -0.0 == +0.0), the lower n/2 members going to box 2b and the rest to
// 2b + 1.  The palette entry of a box is the FP64 mean of its members rounded
// once to FP16; each leaf keeps the uint16 index of its box.
//
// Device layout: the points live in a dense FP32 array [N][D] kept in box
// order (box b occupies positions [start[b], start[b+1])), with the leaf id
// of each position beside it; a round computes per-box min/max per dimension,
// picks the cut dimension, finds each box's median key by an 8-bit-digit radix
// select over 64-bit keys (value bits << LB | leaf id), and scatters the rows
// into the two halves through one global exclusive scan.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dot_device.h"

namespace dot {

namespace {

constexpr int PB = 256;       // threads per workgroup
constexpr int CH = 4096;      // positions per (box, chunk) workgroup

struct Bufs {
    float *X, *X2;
    uint32_t *ids, *ids2, *flags, *lpos, *bsum, *tot;
    uint64_t *keys, *prefix;
    uint32_t *start, *start2, *mm, *hist, *kk;
    int32_t* dim;
};

__device__ __forceinline__ uint32_t ord_f32(float f) {
    if (f == 0.f) f = 0.f;   // -0.0 orders with +0.0
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// FP64 -> FP16 rounded once: an FP32 rounded to odd keeps enough bits for the
// final round-to-nearest-even not to be a double rounding
__device__ __forceinline__ uint16_t f64_to_f16(double x) {
    float f = __double2float_rz(x);
    if ((double)f != x) f = __uint_as_float(__float_as_uint(f) | 1u);
    return f32_to_f16(f);
}

template <int DT>
__global__ void k_pal_gather(const void* __restrict__ sh, int stride, int64_t N, int D, float* __restrict__ X,
                             uint32_t* __restrict__ ids) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N * D; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / D;
        const int d = (int)(i - r * D);
        X[i] = load_sigma<DT>(sh, r * stride + d);   // element decode of the SH plane
        if (d == 0) ids[r] = (uint32_t)r;
    }
}

template <int DT>
__global__ void k_pal_sigma(const void* __restrict__ src, int64_t N, uint16_t* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = f32_to_f16(load_sigma<DT>(src, i));
}

// mm is [nb][D][2]: minima start at all ones, maxima at zero
__global__ void k_pal_mm_init(uint32_t* __restrict__ mm, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        mm[2 * i] = 0xffffffffu;
        mm[2 * i + 1] = 0u;
    }
}

__global__ void k_pal_fill(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// per (box, dimension) min and max of the members, as ordered bits.  Wave w of
// the workgroup takes rows lo + w, lo + w + 4, ...; lane d holds dimension d.
__global__ __launch_bounds__(PB) void k_pal_minmax(const float* __restrict__ X, int D, const uint32_t* __restrict__ start,
                                                   int cpb, uint32_t* __restrict__ mm) {
    __shared__ uint32_t smin[PB / 64][64], smax[PB / 64][64];
    const int b = blockIdx.x / cpb, c = blockIdx.x % cpb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    uint32_t mn = 0xffffffffu, mx = 0u;
    for (int64_t lo = (int64_t)s0 + (int64_t)c * CH; lo < s1; lo += (int64_t)cpb * CH) {
        const int64_t hi = lo + CH < (int64_t)s1 ? lo + CH : (int64_t)s1;
        if (lane < D)
            for (int64_t r = lo + w; r < hi; r += PB / 64) {
                const uint32_t o = ord_f32(X[r * D + lane]);
                mn = min(mn, o);
                mx = max(mx, o);
            }
    }
    smin[w][lane] = mn;
    smax[w][lane] = mx;
    __syncthreads();
    if (w == 0 && lane < D) {
        for (int j = 1; j < PB / 64; ++j) {
            mn = min(mn, smin[j][lane]);
            mx = max(mx, smax[j][lane]);
        }
        if (mn <= mx) {
            atomicMin(&mm[((int64_t)b * D + lane) * 2], mn);
            atomicMax(&mm[((int64_t)b * D + lane) * 2 + 1], mx);
        }
    }
}

// cut dimension of every box (widest max - min in FP64, first of equals) and
// the radix-select state: rank n/2, empty prefix
__global__ void k_pal_dim(const uint32_t* __restrict__ mm, int D, const uint32_t* __restrict__ start, int64_t nb,
                          int32_t* __restrict__ dim, uint64_t* __restrict__ prefix, uint32_t* __restrict__ kk) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t n = start[b + 1] - start[b];
        int best = 0;
        double bw = -1.0;
        if (n > 0)
            for (int d = 0; d < D; ++d) {
                const double w = (double)unord_f32(mm[(b * D + d) * 2 + 1]) - (double)unord_f32(mm[(b * D + d) * 2]);
                if (w > bw) {
                    bw = w;
                    best = d;
                }
            }
        dim[b] = best;
        prefix[b] = 0ull;
        kk[b] = n / 2;
    }
}

__global__ __launch_bounds__(PB) void k_pal_keys(const float* __restrict__ X, int D, const uint32_t* __restrict__ ids,
                                                 const uint32_t* __restrict__ start, int cpb,
                                                 const int32_t* __restrict__ dim, int lb,
                                                 uint64_t* __restrict__ keys) {
    const int b = blockIdx.x / cpb, c = blockIdx.x % cpb;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    const int d = dim[b];
    for (int64_t base = (int64_t)s0 + (int64_t)c * CH; base < s1; base += (int64_t)cpb * CH) {
        const int64_t end = base + CH < (int64_t)s1 ? base + CH : (int64_t)s1;
        for (int64_t i = base + threadIdx.x; i < end; i += PB) keys[i] = ((uint64_t)ord_f32(X[i * D + d]) << lb) | ids[i];
    }
}

// histogram of the current digit over the keys that match the prefix so far
__global__ __launch_bounds__(PB) void k_pal_hist(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ start,
                                                 int cpb, int shift, const uint64_t* __restrict__ prefix,
                                                 uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int b = blockIdx.x / cpb, c = blockIdx.x % cpb;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    const uint64_t pre = prefix[b];
    const int up = shift + 8;
    for (int64_t base = (int64_t)s0 + (int64_t)c * CH; base < s1; base += (int64_t)cpb * CH) {
        const int64_t end = base + CH < (int64_t)s1 ? base + CH : (int64_t)s1;
        for (int64_t i = base + threadIdx.x; i < end; i += PB) {
            const uint64_t k = keys[i];
            if (up >= 64 || (k >> up) == (pre >> up)) atomicAdd(&h[(k >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[(int64_t)b * 256 + threadIdx.x], h[threadIdx.x]);
}

// one wave per box: the digit holding rank kk, appended to the prefix; the
// box's histogram is cleared for the next digit
__global__ void k_pal_digit(uint32_t* __restrict__ hist, const uint32_t* __restrict__ start, int64_t nb, int shift,
                            uint64_t* __restrict__ prefix, uint32_t* __restrict__ kk) {
    const int64_t b = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= nb) return;
    uint32_t* h = hist + b * 256;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = h[lane * 4 + j];
        sum += v[j];
    }
    // inclusive scan of the lane sums
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    const uint32_t excl = incl - sum;
    const uint32_t k = kk[b];
    const bool has = start[b + 1] > start[b];
    // the lane whose bins contain rank k
    if (has && k >= excl && k < incl) {
        uint32_t acc = excl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (k < acc + v[j]) {
                prefix[b] |= (uint64_t)(lane * 4 + j) << shift;
                kk[b] = k - acc;
                break;
            }
            acc += v[j];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) h[lane * 4 + j] = 0u;
}

__global__ __launch_bounds__(PB) void k_pal_flags(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ start,
                                                  int cpb, const uint64_t* __restrict__ kth,
                                                  uint32_t* __restrict__ flags) {
    const int b = blockIdx.x / cpb, c = blockIdx.x % cpb;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    const uint64_t m = kth[b];
    for (int64_t base = (int64_t)s0 + (int64_t)c * CH; base < s1; base += (int64_t)cpb * CH) {
        const int64_t end = base + CH < (int64_t)s1 ? base + CH : (int64_t)s1;
        for (int64_t i = base + threadIdx.x; i < end; i += PB) flags[i] = keys[i] < m ? 1u : 0u;
    }
}

// move every member to its half: lower members keep their order at the front
// of the box, upper members theirs behind them
__global__ __launch_bounds__(PB) void k_pal_scatter(const float* __restrict__ X, const uint32_t* __restrict__ ids, int D,
                                                    const uint32_t* __restrict__ start, int cpb,
                                                    const uint32_t* __restrict__ flags,
                                                    const uint32_t* __restrict__ lpos, float* __restrict__ X2,
                                                    uint32_t* __restrict__ ids2) {
    const int b = blockIdx.x / cpb, c = blockIdx.x % cpb;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    if (s0 >= s1) return;
    const uint32_t half = (s1 - s0) / 2, base = lpos[s0];
    for (int64_t cb = (int64_t)s0 + (int64_t)c * CH; cb < s1; cb += (int64_t)cpb * CH) {
        const int64_t end = cb + CH < (int64_t)s1 ? cb + CH : (int64_t)s1;
        for (int64_t i = cb + threadIdx.x; i < end; i += PB) {
            const uint32_t li = lpos[i] - base;
            int64_t dst = flags[i] ? (int64_t)s0 + li : (int64_t)s0 + half + (i - s0) - li;
            // exactly `half` members are flagged (the keys are distinct), so dst
            // stays in the box; the clamp only keeps a broken invariant in bounds
            dst = dst < (int64_t)s0 ? (int64_t)s0 : (dst >= (int64_t)s1 ? (int64_t)s1 - 1 : dst);
            const float* src = X + i * D;
            float* o = X2 + dst * D;
            for (int d = 0; d < D; ++d) o[d] = src[d];
            ids2[dst] = ids[i];
        }
    }
}

__global__ void k_pal_starts(const uint32_t* __restrict__ start, int64_t nb, uint32_t* __restrict__ start2) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        start2[2 * b] = start[b];
        start2[2 * b + 1] = start[b] + (start[b + 1] - start[b]) / 2;
        if (b == nb - 1) start2[2 * nb] = start[nb];
    }
}

// one wave per box: lane d sums dimension d in FP64 in position order; the
// mean rounded once to FP16; every member's leaf gets the box index
__global__ void k_pal_mean(const float* __restrict__ X, const uint32_t* __restrict__ ids, int D, int pstride,
                           const uint32_t* __restrict__ start, int64_t nb, uint16_t* __restrict__ pal,
                           uint16_t* __restrict__ index) {
    const int64_t b = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= nb) return;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    if (lane < pstride) {
        uint16_t out = 0;
        if (lane < D && s1 > s0) {
            double acc = 0.0;
            for (uint32_t r = s0; r < s1; ++r) acc += (double)X[(int64_t)r * D + lane];
            out = f64_to_f16(acc / (double)(s1 - s0));
        }
        pal[b * pstride + lane] = out;
    }
    for (uint32_t r = s0 + lane; r < s1; r += 64) index[ids[r]] = (uint16_t)b;
}

unsigned g1(int64_t n) {
    int64_t g = (n + PB - 1) / PB;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}

}  // namespace

// dst[r][d] = palette[index[row0 + r]][d] for rows [row0, row0 + rows), FP32
__global__ void k_pal_decode(const uint16_t* __restrict__ index, const uint16_t* __restrict__ pal, int pstride, int D,
                             int64_t rows, int64_t row0, float* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows * D; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / D;
        const int d = (int)(i - r * D);
        dst[i] = f16_to_f32(pal[(int64_t)index[row0 + r] * pstride + d]);
    }
}

hipError_t launch_decode_palette(const dot_tree& t, float* dst, int64_t rows, int64_t row0, hipStream_t s) {
    if (rows == 0) return hipSuccess;
    const int D = 3 * (t.degree + 1) * (t.degree + 1);
    hipLaunchKernelGGL(k_pal_decode, dim3(g1(rows * D)), dim3(PB), 0, s, static_cast<const uint16_t*>(t.sh),
                       static_cast<const uint16_t*>(t.palette), t.sh_stride, D, rows, row0, dst);
    return hipGetLastError();
}

int quantize_sh(dot_tree& t, int bits, hipStream_t s) {
    const int64_t N = t.n_leaves;
    const int D = 3 * (t.degree + 1) * (t.degree + 1);
    const int64_t P = (int64_t)1 << bits;
    const int pstride = sh_stride_for(t.degree, DOT_F16);
    int lb = 1;
    while (((int64_t)1 << lb) < N) ++lb;
    const Alloc& al = t.alloc;
    // scratch
    struct Owned {
        const Alloc& al;
        void* p[24] = {};
        int n = 0;
        explicit Owned(const Alloc& a) : al(a) {}
        void* get(size_t bytes) {
            void* q = al.get(bytes);
            p[n++] = q;
            return q;
        }
        bool ok() const {
            for (int i = 0; i < n; ++i)
                if (!p[i]) return false;
            return true;
        }
        ~Owned() {
            for (int i = 0; i < n; ++i) al.put(p[i]);
        }
    } tmp(al);
    const int64_t nbmax = P / 2;
    Bufs B;
    B.X = static_cast<float*>(tmp.get((size_t)N * D * 4));
    B.X2 = static_cast<float*>(tmp.get((size_t)N * D * 4));
    B.ids = static_cast<uint32_t*>(tmp.get((size_t)N * 4));
    B.ids2 = static_cast<uint32_t*>(tmp.get((size_t)N * 4));
    B.flags = static_cast<uint32_t*>(tmp.get((size_t)N * 4));
    B.lpos = static_cast<uint32_t*>(tmp.get((size_t)N * 4));
    B.bsum = static_cast<uint32_t*>(tmp.get((size_t)scan_scratch_elems(N) * 4));
    B.tot = static_cast<uint32_t*>(tmp.get(16));
    B.keys = static_cast<uint64_t*>(tmp.get((size_t)N * 8));
    B.prefix = static_cast<uint64_t*>(tmp.get((size_t)nbmax * 8));
    B.start = static_cast<uint32_t*>(tmp.get((size_t)(P + 1) * 4));
    B.start2 = static_cast<uint32_t*>(tmp.get((size_t)(P + 1) * 4));
    B.mm = static_cast<uint32_t*>(tmp.get((size_t)nbmax * D * 2 * 4));
    B.hist = static_cast<uint32_t*>(tmp.get((size_t)nbmax * 256 * 4));
    B.kk = static_cast<uint32_t*>(tmp.get((size_t)nbmax * 4));
    B.dim = static_cast<int32_t*>(tmp.get((size_t)nbmax * 4));
    // the new planes
    uint16_t* sig16 = static_cast<uint16_t*>(al.get((size_t)N * 2));
    uint16_t* index = static_cast<uint16_t*>(al.get((size_t)N * 2));
    uint16_t* pal = static_cast<uint16_t*>(al.get((size_t)P * pstride * 2));
    auto drop_new = [&]() {
        al.put(sig16);
        al.put(index);
        al.put(pal);
    };
    if (!tmp.ok() || !sig16 || !index || !pal) {
        drop_new();
        return fail(DOT_ENOMEM, "dot_quantize_sh: scratch allocation failed");
    }
    hipError_t e = hipSuccess;
    switch (t.storage) {
        case DOT_F32:
            hipLaunchKernelGGL(k_pal_gather<DOT_F32>, dim3(g1(N * D)), dim3(PB), 0, s, t.sh, t.sh_stride, N, D, B.X, B.ids);
            hipLaunchKernelGGL(k_pal_sigma<DOT_F32>, dim3(g1(N)), dim3(PB), 0, s, t.sigma, N, sig16);
            break;
        case DOT_F16:
            hipLaunchKernelGGL(k_pal_gather<DOT_F16>, dim3(g1(N * D)), dim3(PB), 0, s, t.sh, t.sh_stride, N, D, B.X, B.ids);
            hipLaunchKernelGGL(k_pal_sigma<DOT_F16>, dim3(g1(N)), dim3(PB), 0, s, t.sigma, N, sig16);
            break;
        default:
            hipLaunchKernelGGL(k_pal_gather<DOT_BF16>, dim3(g1(N * D)), dim3(PB), 0, s, t.sh, t.sh_stride, N, D, B.X, B.ids);
            hipLaunchKernelGGL(k_pal_sigma<DOT_BF16>, dim3(g1(N)), dim3(PB), 0, s, t.sigma, N, sig16);
            break;
    }
    // start = {0, N}
    const uint32_t init[2] = {0u, (uint32_t)N};
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(B.start, init, sizeof(init), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // `init` is on the host stack
    const int nd = (32 + lb + 7) / 8;                  // digits of a key
    for (int r = 0; r < bits && e == hipSuccess; ++r) {
        const int64_t nb = (int64_t)1 << r;
        const int64_t maxn = (N + nb - 1) / nb;
        const int cpb = (int)std::max<int64_t>(1, (maxn + CH - 1) / CH);
        const unsigned grid = (unsigned)(nb * cpb);
        hipLaunchKernelGGL(k_pal_mm_init, dim3(g1(nb * D)), dim3(PB), 0, s, B.mm, nb * D);
        hipLaunchKernelGGL(k_pal_fill, dim3(g1(nb * 256)), dim3(PB), 0, s, B.hist, nb * 256, 0u);
        hipLaunchKernelGGL(k_pal_minmax, dim3(grid), dim3(PB), 0, s, B.X, D, B.start, cpb, B.mm);
        hipLaunchKernelGGL(k_pal_dim, dim3(g1(nb)), dim3(PB), 0, s, B.mm, D, B.start, nb, B.dim, B.prefix, B.kk);
        hipLaunchKernelGGL(k_pal_keys, dim3(grid), dim3(PB), 0, s, B.X, D, B.ids, B.start, cpb, B.dim, lb, B.keys);
        for (int p = 0; p < nd; ++p) {
            const int shift = (nd - 1 - p) * 8;
            hipLaunchKernelGGL(k_pal_hist, dim3(grid), dim3(PB), 0, s, B.keys, B.start, cpb, shift, B.prefix, B.hist);
            hipLaunchKernelGGL(k_pal_digit, dim3((unsigned)((nb + 3) / 4)), dim3(PB), 0, s, B.hist, B.start, nb, shift,
                               B.prefix, B.kk);
        }
        hipLaunchKernelGGL(k_pal_flags, dim3(grid), dim3(PB), 0, s, B.keys, B.start, cpb, B.prefix, B.flags);
        e = hipGetLastError();
        if (e == hipSuccess) e = scan_u32(B.flags, B.lpos, N, B.bsum, B.tot, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_pal_scatter, dim3(grid), dim3(PB), 0, s, B.X, B.ids, D, B.start, cpb, B.flags, B.lpos,
                           B.X2, B.ids2);
        hipLaunchKernelGGL(k_pal_starts, dim3(g1(nb)), dim3(PB), 0, s, B.start, nb, B.start2);
        e = hipGetLastError();
        std::swap(B.X, B.X2);
        std::swap(B.ids, B.ids2);
        std::swap(B.start, B.start2);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pal_mean, dim3((unsigned)((P + 3) / 4)), dim3(PB), 0, s, B.X, B.ids, D, pstride, B.start,
                           P, pal, index);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        drop_new();
        return hip_fail(e, "dot_quantize_sh");
    }
    al.put(t.sigma);
    al.put(t.sh);
    t.sigma = sig16;
    t.sh = index;
    t.palette = pal;
    t.palette_bits = bits;
    t.storage = DOT_PAL16;
    t.sh_stride = pstride;
    return DOT_OK;
}

}  // namespace dot
