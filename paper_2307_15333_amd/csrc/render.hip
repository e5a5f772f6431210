// Forward renderer (Eq. 1-2 with the fused training signal) and its adjoint.
#include <hip/hip_runtime.h>

#include "dot_device.h"

namespace dot {

template <int DT, int DEG, bool STATS>
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
    FwdSeg<DT, DEG> seg(tv, a);
    sh_basis<DEG>((float)r.dx, (float)r.dy, (float)r.dz, seg.Y);
    int desc = 0;
    traverse(tv, r, &stack_lds[tid], seg, desc);
    if (a.rgb) {
        float Te = seg.T;
        a.rgb[3 * rid + 0] = fmaf(Te, a.bg[0], seg.C[0]);
        a.rgb[3 * rid + 1] = fmaf(Te, a.bg[1], seg.C[1]);
        a.rgb[3 * rid + 2] = fmaf(Te, a.bg[2], seg.C[2]);
    }
    if (a.nseg) a.nseg[rid] = seg.n;
    if constexpr (STATS) {
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

template <int DT, int DEG>
static hipError_t fwd_dispatch_stats(const TreeView& tv, const RayBatch& rb, const FwdArgs& a,
                                     dim3 grid, hipStream_t s) {
    if (a.stats)
        hipLaunchKernelGGL((render_fwd_kernel<DT, DEG, true>), grid, dim3(BLOCK), 0, s, tv, rb, a);
    else
        hipLaunchKernelGGL((render_fwd_kernel<DT, DEG, false>), grid, dim3(BLOCK), 0, s, tv, rb, a);
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

hipError_t launch_render_bwd(const dot_tree& t, const RayBatch& rb, const BwdArgs& a, hipStream_t s) {
    if (rb.n_tiles == 0) return hipSuccess;
    dim3 grid((unsigned)((rb.n_tiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
    TreeView tv = t.view();
    switch (t.storage) {
        case DOT_F32: return bwd_dispatch_deg<DOT_F32>(t.degree, tv, rb, a, grid, s);
        case DOT_F16: return bwd_dispatch_deg<DOT_F16>(t.degree, tv, rb, a, grid, s);
        default: return bwd_dispatch_deg<DOT_BF16>(t.degree, tv, rb, a, grid, s);
    }
}

}  // namespace dot
