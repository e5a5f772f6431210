// Octree refinement on the device (Sec. 3.2, Alg. 1: pruning, then sampling,
// both driven by the same per-leaf signal).
//
//   mark    an internal node merges iff its 8 children are leaves and all are
//           selected for pruning (signal <= tau, or < tau); with recursive
//           pruning (the paper's "(R)" option) merging repeats up the
//           hierarchy, which ends with every node whose subtree leaves are all
//           selected merged: the subtree's leaves are a contiguous DFS range,
//           so one prefix count of unselected leaves decides every node;
//   select  exact top-k of the 64-bit keys (~ord(signal) << 32 | leaf) over
//           the sampling candidates by an 8-pass MSD radix select, so ties in
//           signal go to the lower leaf index;
//   rebuild new leaf and internal indices by exclusive prefix scans over the
//           old DFS order, then scatter: a merged group becomes one leaf with
//           the mean of its 8 rows (Eq. 3), a sampled leaf becomes an internal
//           node whose 8 children copy its row (Eq. 4).
// The result is numbered in DFS order, so its topology is canonical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dot_device.h"

namespace dot {

namespace {

constexpr int TPB = 256;

unsigned blocks_for(int64_t n, int per_thread = 1) {
    int64_t g = (n + (int64_t)TPB * per_thread - 1) / ((int64_t)TPB * per_thread);
    if (g > 1 << 20) g = 1 << 20;
    return (unsigned)(g < 1 ? 1 : g);
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ bool selected(float s, float tau, int le) { return le ? (s <= tau) : (s < tau); }

// order-preserving map of a float to uint32 (ascending)
__device__ __forceinline__ uint32_t ord32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    GRID_STRIDE(i, n) p[i] = v;
}

// first / last leaf of each internal node's subtree and the node's depth
__global__ void k_node_meta(const int32_t* __restrict__ child, int64_t I, const uint8_t* __restrict__ leaf_depth,
                            int32_t* __restrict__ first, int32_t* __restrict__ last, int32_t* __restrict__ ndepth) {
    GRID_STRIDE(p, I) {
        int steps = 1;
        int32_t e = child[p * 8];
        while (e >= 0) {
            e = child[(int64_t)e * 8];
            ++steps;
        }
        first[p] = -1 - e;
        ndepth[p] = (int32_t)leaf_depth[-1 - e] - steps;
        e = child[p * 8 + 7];
        while (e >= 0) e = child[(int64_t)e * 8 + 7];
        last[p] = -1 - e;
    }
}

__global__ void k_node_parent(const int32_t* __restrict__ child, int64_t I, int32_t* __restrict__ parent) {
    GRID_STRIDE(j, I * 8) {
        int32_t e = child[j];
        if (e >= 0) parent[e] = (int32_t)(j >> 3);
    }
}

__global__ void k_unselected(const float* __restrict__ sig, int64_t L, float tau, int le, uint32_t* __restrict__ u) {
    GRID_STRIDE(l, L) u[l] = selected(sig[l], tau, le) ? 0u : 1u;
}

// merge roots and survivors.  all_sel[p]: no unselected leaf in [first, last].
__global__ void k_mark_merge(const int32_t* __restrict__ child, int64_t I, const int32_t* __restrict__ first,
                             const int32_t* __restrict__ last, const int32_t* __restrict__ parent,
                             const uint32_t* __restrict__ unsel, const uint32_t* __restrict__ pre_unsel,
                             int recursive, uint32_t* __restrict__ survive, uint32_t* __restrict__ root,
                             uint32_t* __restrict__ need) {
    GRID_STRIDE(p, I) {
        auto all_sel = [&](int64_t q) {
            int32_t f = first[q], l = last[q];
            return pre_unsel[l] + unsel[l] - pre_unsel[f] == 0u;
        };
        bool as = all_sel(p);
        bool r;
        if (recursive) {
            r = as && (p == 0 || !all_sel(parent[p]));
            survive[p] = as ? 0u : 1u;
            need[p] = as ? 1u : 0u;
        } else {
            bool leaves = true;
#pragma unroll
            for (int o = 0; o < 8; ++o) leaves &= child[p * 8 + o] < 0;
            r = as && leaves;
            survive[p] = r ? 0u : 1u;
            need[p] = r ? 1u : 0u;
        }
        root[p] = r ? 1u : 0u;
    }
}

// every leaf under a merge root records the root (roots' ranges are disjoint)
__global__ void k_cover(int64_t I, const uint32_t* __restrict__ root, const int32_t* __restrict__ first,
                        const int32_t* __restrict__ last, int32_t* __restrict__ cover) {
    GRID_STRIDE(p, I) {
        if (!root[p]) continue;
        for (int32_t l = first[p]; l <= last[p]; ++l) cover[l] = (int32_t)p;
    }
}

__global__ void k_keys(const float* __restrict__ sig, const uint8_t* __restrict__ depth, int64_t L, float tau,
                       int le, int max_depth, uint64_t* __restrict__ keys) {
    GRID_STRIDE(l, L) {
        float s = sig[l];
        bool cand = !selected(s, tau, le) && (int)depth[l] < max_depth;
        keys[l] = cand ? (((uint64_t)(~ord32(s)) << 32) | (uint64_t)l) : ~0ull;
    }
}

struct SelState {
    unsigned long long prefix, mask;
    unsigned long long k_rem, k_eff;
    unsigned int hist[256];
};

__global__ void k_sel_init(SelState* st) {
    int t = threadIdx.x;
    if (t == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->k_rem = 0;
        st->k_eff = 0;
    }
    st->hist[t] = 0;
}

__global__ void k_hist(const uint64_t* __restrict__ keys, int64_t L, int shift, SelState* st) {
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const unsigned long long prefix = st->prefix, mask = st->mask;
    GRID_STRIDE(l, L) {
        uint64_t k = keys[l];
        if (k != ~0ull && (k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}

// one thread: choose the digit holding the k_rem-th smallest candidate
__global__ void k_sel_digit(SelState* st, int shift, int first, long long k_req) {
    if (threadIdx.x != 0) return;
    if (first) {
        unsigned long long n = 0;
        for (int d = 0; d < 256; ++d) n += st->hist[d];
        unsigned long long k = (unsigned long long)k_req < n ? (unsigned long long)k_req : n;
        st->k_eff = k;
        st->k_rem = k;
    }
    if (st->k_rem > 0) {
        unsigned long long cum = 0;
        int d = 0;
        for (; d < 256; ++d) {
            if (cum + st->hist[d] >= st->k_rem) break;
            cum += st->hist[d];
        }
        st->k_rem -= cum;
        st->prefix |= (unsigned long long)d << shift;
        st->mask |= 255ull << shift;
    }
    for (int d = 0; d < 256; ++d) st->hist[d] = 0;
}

// new-leaf counts per old leaf, and the split flags
__global__ void k_leaf_counts(int64_t L, const int32_t* __restrict__ cover, const int32_t* __restrict__ first,
                              const uint64_t* __restrict__ keys, const SelState* __restrict__ st,
                              uint32_t* __restrict__ cnt, uint32_t* __restrict__ split) {
    const unsigned long long kstar = st->prefix;
    const bool any = st->k_eff > 0;
    GRID_STRIDE(l, L) {
        int32_t c = cover[l];
        bool sp = any && keys[l] != ~0ull && keys[l] <= kstar;
        split[l] = sp ? 1u : 0u;
        cnt[l] = c >= 0 ? (first[c] == (int32_t)l ? 1u : 0u) : (sp ? 8u : 1u);
    }
}

__global__ void k_add_u32(uint32_t* __restrict__ a, const uint32_t* __restrict__ h, int64_t n) {
    GRID_STRIDE(i, n) a[i] += h[i];
}

__global__ void k_first_hist(int64_t I, const uint32_t* __restrict__ survive, const int32_t* __restrict__ first,
                             uint32_t* __restrict__ hist) {
    GRID_STRIDE(p, I) {
        if (survive[p]) atomicAdd(&hist[first[p]], 1u);
    }
}

// ---- rebuild ----
__global__ void k_child_internal(const int32_t* __restrict__ child, int64_t I, const uint32_t* __restrict__ survive,
                                 const int32_t* __restrict__ first, const uint32_t* __restrict__ rank_int,
                                 const uint32_t* __restrict__ rank_split, const uint32_t* __restrict__ split,
                                 const uint32_t* __restrict__ cnt_le, const uint32_t* __restrict__ nl,
                                 int32_t* __restrict__ out) {
    GRID_STRIDE(p, I) {
        if (!survive[p]) continue;
        int64_t np = (int64_t)rank_int[p] + rank_split[first[p]];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            int32_t e = child[p * 8 + o];
            int32_t v;
            if (e >= 0) {
                if (survive[e])
                    v = (int32_t)(rank_int[e] + rank_split[first[e]]);
                else
                    v = -1 - (int32_t)nl[first[e]];
            } else {
                int64_t l = -1 - e;
                if (split[l])
                    v = (int32_t)(rank_split[l] + cnt_le[l]);
                else
                    v = -1 - (int32_t)nl[l];
            }
            out[np * 8 + o] = v;
        }
    }
}

__global__ void k_child_split(int64_t L, const uint32_t* __restrict__ split, const uint32_t* __restrict__ rank_split,
                              const uint32_t* __restrict__ cnt_le, const uint32_t* __restrict__ nl,
                              int32_t* __restrict__ out) {
    GRID_STRIDE(l, L) {
        if (!split[l]) continue;
        int64_t np = (int64_t)rank_split[l] + cnt_le[l];
#pragma unroll
        for (int o = 0; o < 8; ++o) out[np * 8 + o] = -1 - (int32_t)(nl[l] + o);
    }
}

template <int DT>
__device__ __forceinline__ double ld_elem(const void* p, int64_t i) {
    if constexpr (DT == DOT_F32)
        return (double)static_cast<const float*>(p)[i];
    else if constexpr (DT == DOT_F16)
        return (double)f16_to_f32(static_cast<const uint16_t*>(p)[i]);
    else
        return (double)bf16_to_f32(static_cast<const uint16_t*>(p)[i]);
}

// FP64 -> storage, round to nearest even, rounded once: FP32 directly; FP16 /
// BF16 through an FP32 rounded to odd (truncate, set the last bit if inexact),
// which carries enough bits that the final rounding is not a double rounding.
template <int DT>
__device__ __forceinline__ void st_elem(void* p, int64_t i, double x) {
    if constexpr (DT == DOT_F32) {
        static_cast<float*>(p)[i] = __double2float_rn(x);
    } else {
        float f = __double2float_rz(x);
        if ((double)f != x) f = __uint_as_float(__float_as_uint(f) | 1u);
        static_cast<uint16_t*>(p)[i] = DT == DOT_F16 ? f32_to_f16(f) : f32_to_bf16(f);
    }
}

template <int DT>
__device__ __forceinline__ void cp_elem(const void* src, int64_t i, void* dst, int64_t j) {
    if constexpr (DT == DOT_F32)
        static_cast<float*>(dst)[j] = static_cast<const float*>(src)[i];
    else
        static_cast<uint16_t*>(dst)[j] = static_cast<const uint16_t*>(src)[i];
}

// Values of merged nodes, one depth level per launch from the deepest up: the
// mean of the 8 children's rows (leaf rows, or node rows formed by the previous
// launch), summed pairwise in FP64 and rounded once to the storage type.
// Row layout of nval: [sigma, sh[0..stride)] per node, in the storage type.
template <int DT>
__global__ void k_node_values(const int32_t* __restrict__ child, int64_t I, int depth,
                              const int32_t* __restrict__ ndepth, const uint32_t* __restrict__ need, int nv,
                              int stride, const void* __restrict__ sig, const void* __restrict__ sh,
                              void* __restrict__ nval) {
    const int row = stride + 1;
    GRID_STRIDE(p, I) {
        if (!need[p] || ndepth[p] != depth) continue;
        int32_t e[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) e[o] = child[p * 8 + o];
        for (int c = -1; c < nv; ++c) {
            double v[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                if (e[o] < 0) {
                    int64_t l = -1 - e[o];
                    v[o] = c < 0 ? ld_elem<DT>(sig, l) : ld_elem<DT>(sh, l * stride + c);
                } else {
                    v[o] = ld_elem<DT>(nval, (int64_t)e[o] * row + 1 + c);
                }
            }
            double m = (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) * 0.125;
            st_elem<DT>(nval, p * row + 1 + c, m);
        }
        for (int c = nv; c < stride; ++c) st_elem<DT>(nval, p * row + 1 + c, 0.0);
    }
}

template <int DT>
__global__ void k_emit_leaves(int64_t L, int stride, int reinit, const int32_t* __restrict__ cover,
                              const int32_t* __restrict__ first, const int32_t* __restrict__ ndepth,
                              const uint32_t* __restrict__ split, const uint32_t* __restrict__ nl,
                              const uint8_t* __restrict__ depth, const void* __restrict__ sig,
                              const void* __restrict__ sh, const void* __restrict__ nval, void* __restrict__ sig2,
                              void* __restrict__ sh2, uint8_t* __restrict__ depth2) {
    const int row = stride + 1;
    GRID_STRIDE(l, L) {
        int32_t c = cover[l];
        int64_t j = nl[l];
        if (c >= 0) {
            if (first[c] != (int32_t)l) continue;
            if (reinit) {
                st_elem<DT>(sig2, j, 0.0);
                for (int k = 0; k < stride; ++k) st_elem<DT>(sh2, j * stride + k, 0.0);
            } else {
                cp_elem<DT>(nval, (int64_t)c * row, sig2, j);
                for (int k = 0; k < stride; ++k) cp_elem<DT>(nval, (int64_t)c * row + 1 + k, sh2, j * stride + k);
            }
            depth2[j] = (uint8_t)ndepth[c];
        } else {
            int reps = split[l] ? 8 : 1;
            uint8_t d = (uint8_t)(depth[l] + (split[l] ? 1 : 0));
            for (int r = 0; r < reps; ++r) {
                if (reinit && split[l]) {
                    st_elem<DT>(sig2, j + r, 0.0);
                    for (int k = 0; k < stride; ++k) st_elem<DT>(sh2, (j + r) * stride + k, 0.0);
                } else {
                    cp_elem<DT>(sig, l, sig2, j + r);
                    for (int k = 0; k < stride; ++k) cp_elem<DT>(sh, l * stride + k, sh2, (j + r) * stride + k);
                }
                depth2[j + r] = d;
            }
        }
    }
}

__global__ void k_totals(int64_t L, int64_t I, const uint32_t* __restrict__ nl, const uint32_t* __restrict__ cnt,
                         const uint32_t* __restrict__ tot_int, const uint32_t* __restrict__ tot_split,
                         const SelState* __restrict__ st, unsigned long long* __restrict__ out) {
    if (threadIdx.x != 0) return;
    out[0] = (unsigned long long)nl[L - 1] + cnt[L - 1];      // new leaves
    out[1] = (unsigned long long)(I > 0 ? *tot_int : 0u) + *tot_split;  // new internal nodes
    out[2] = (unsigned long long)(I > 0 ? (uint64_t)I - *tot_int : 0u);  // merged nodes
    out[3] = st->k_eff;
}

// RAII list of temporaries from the tree's allocator
struct Temps {
    const Alloc& al;
    std::vector<void*> ps;
    bool ok = true;
    explicit Temps(const Alloc& a) : al(a) {}
    template <class T>
    T* get(int64_t n) {
        void* p = al.get((size_t)(n < 1 ? 1 : n) * sizeof(T));
        if (!p) ok = false;
        ps.push_back(p);
        return static_cast<T*>(p);
    }
    ~Temps() {
        for (void* p : ps) al.put(p);
    }
};

template <int DT>
hipError_t launch_values_emit(const dot_tree& t, int64_t L, int64_t I, int nv, int stride, int reinit,
                              const int32_t* cover,
                              const int32_t* first, const int32_t* ndepth, const uint32_t* need,
                              const uint32_t* split, const uint32_t* nl, void* nval, void* sig2, void* sh2,
                              uint8_t* depth2, hipStream_t s) {
    if (I > 0)
        for (int d = DOT_MAX_DEPTH - 1; d >= 0; --d)
            hipLaunchKernelGGL(k_node_values<DT>, dim3(blocks_for(I)), dim3(TPB), 0, s, t.child, I, d, ndepth, need,
                               nv, stride, t.sigma, t.sh, nval);
    hipLaunchKernelGGL(k_emit_leaves<DT>, dim3(blocks_for(L)), dim3(TPB), 0, s, L, stride, reinit, cover, first, ndepth,
                       split,
                       nl, t.leaf_depth, t.sigma, t.sh, nval, sig2, sh2, depth2);
    return hipGetLastError();
}

}  // namespace

int refine_tree(dot_tree& t, const float* signal, const dot_refine_params& p, dot_refine_stats* st_out,
                hipStream_t s) {
    const int64_t L = t.n_leaves, I = t.n_internal;
    const int64_t k_req = (int64_t)std::floor((double)p.sample_frac * (double)L);
    if (L + 7 * k_req > (int64_t)INT32_MAX || I + k_req > (int64_t)INT32_MAX / 8)
        return fail(DOT_EINVAL, "dot_refine: the refined tree would exceed 32-bit indices");
    const int nv = 3 * (t.degree + 1) * (t.degree + 1);
    const int stride = t.sh_stride;
    const int es = storage_bytes(t.storage);
    const int rec = p.recursive ? 1 : 0;

    Temps tmp(t.alloc);
    int32_t* first = tmp.get<int32_t>(I);
    int32_t* last = tmp.get<int32_t>(I);
    int32_t* ndepth = tmp.get<int32_t>(I);
    int32_t* parent = tmp.get<int32_t>(I);
    uint32_t* survive = tmp.get<uint32_t>(I);
    uint32_t* root = tmp.get<uint32_t>(I);
    uint32_t* need = tmp.get<uint32_t>(I);
    uint32_t* rank_int = tmp.get<uint32_t>(I);
    void* nval = tmp.get<unsigned char>(std::max<int64_t>(I, 1) * (stride + 1) * es);
    uint32_t* unsel = tmp.get<uint32_t>(L);
    uint32_t* pre_unsel = tmp.get<uint32_t>(L);
    int32_t* cover = tmp.get<int32_t>(L);
    uint64_t* keys = tmp.get<uint64_t>(L);
    SelState* sel = tmp.get<SelState>(1);
    uint32_t* cnt = tmp.get<uint32_t>(L);
    uint32_t* split = tmp.get<uint32_t>(L);
    uint32_t* nl = tmp.get<uint32_t>(L);
    uint32_t* rank_split = tmp.get<uint32_t>(L);
    uint32_t* hist_first = tmp.get<uint32_t>(L);
    uint32_t* cnt_le = tmp.get<uint32_t>(L);
    uint32_t* bsum = tmp.get<uint32_t>(scan_scratch_elems(std::max(L, I)));
    uint32_t* tots = tmp.get<uint32_t>(8);
    unsigned long long* totals = tmp.get<unsigned long long>(4);
    if (!tmp.ok) return fail(DOT_ENOMEM, "dot_refine: scratch allocation failed");

    // 1. tree metadata, merge marks, candidate keys
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(L)), dim3(TPB), 0, s, reinterpret_cast<uint32_t*>(cover), L,
                       0xffffffffu);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(L)), dim3(TPB), 0, s, hist_first, L, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(TPB), 0, s, tots, (int64_t)8, 0u);
    hipLaunchKernelGGL(k_unselected, dim3(blocks_for(L)), dim3(TPB), 0, s, signal, L, p.prune_tau, p.prune_le, unsel);
    hipError_t e = scan_u32(unsel, pre_unsel, L, bsum, &tots[4], s);
    if (e != hipSuccess) return hip_fail(e, "dot_refine: scan");
    if (I > 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(TPB), 0, s, reinterpret_cast<uint32_t*>(parent), (int64_t)1,
                           0xffffffffu);
        hipLaunchKernelGGL(k_node_parent, dim3(blocks_for(I * 8)), dim3(TPB), 0, s, t.child, I, parent);
        hipLaunchKernelGGL(k_node_meta, dim3(blocks_for(I)), dim3(TPB), 0, s, t.child, I, t.leaf_depth, first, last,
                           ndepth);
        hipLaunchKernelGGL(k_mark_merge, dim3(blocks_for(I)), dim3(TPB), 0, s, t.child, I, first, last, parent, unsel,
                           pre_unsel, rec, survive, root, need);
        hipLaunchKernelGGL(k_cover, dim3(blocks_for(I)), dim3(TPB), 0, s, I, root, first, last, cover);
    }
    hipLaunchKernelGGL(k_keys, dim3(blocks_for(L)), dim3(TPB), 0, s, signal, t.leaf_depth, L, p.prune_tau,
                       p.prune_le, p.max_depth, keys);
    // 2. exact top-k by radix select over the 64-bit keys
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, sel);
    if (k_req > 0) {
        for (int pass = 0; pass < 8; ++pass) {
            int shift = 56 - 8 * pass;
            hipLaunchKernelGGL(k_hist, dim3(blocks_for(L, 8)), dim3(256), 0, s, keys, L, shift, sel);
            hipLaunchKernelGGL(k_sel_digit, dim3(1), dim3(64), 0, s, sel, shift, pass == 0 ? 1 : 0,
                               (long long)k_req);
        }
    }
    // 3. counts and scans
    hipLaunchKernelGGL(k_leaf_counts, dim3(blocks_for(L)), dim3(TPB), 0, s, L, cover, first, keys, sel, cnt, split);
    if (I > 0) hipLaunchKernelGGL(k_first_hist, dim3(blocks_for(I)), dim3(TPB), 0, s, I, survive, first, hist_first);
    e = scan_u32(cnt, nl, L, bsum, &tots[0], s);
    if (e == hipSuccess) e = scan_u32(split, rank_split, L, bsum, &tots[1], s);
    if (e == hipSuccess) e = scan_u32(hist_first, cnt_le, L, bsum, &tots[2], s);
    if (e == hipSuccess && I > 0) e = scan_u32(survive, rank_int, I, bsum, &tots[3], s);
    if (e != hipSuccess) return hip_fail(e, "dot_refine: scans");
    // cnt_le becomes inclusive: surviving nodes whose first leaf is <= l
    hipLaunchKernelGGL(k_add_u32, dim3(blocks_for(L)), dim3(TPB), 0, s, cnt_le, (const uint32_t*)hist_first, L);
    hipLaunchKernelGGL(k_totals, dim3(1), dim3(64), 0, s, L, I, nl, cnt, &tots[3], &tots[1], sel, totals);
    unsigned long long h_tot[4];
    e = hipMemcpyAsync(h_tot, totals, sizeof(h_tot), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "dot_refine: sizes");
    const int64_t L2 = (int64_t)h_tot[0], I2 = (int64_t)h_tot[1];

    // 4. new planes
    int32_t* child2 = static_cast<int32_t*>(t.alloc.get((size_t)std::max<int64_t>(I2, 1) * 32));
    void* sig2 = t.alloc.get((size_t)L2 * es);
    void* sh2 = t.alloc.get((size_t)L2 * stride * es);
    uint8_t* depth2 = static_cast<uint8_t*>(t.alloc.get((size_t)L2));
    auto drop_new = [&]() {
        t.alloc.put(child2);
        t.alloc.put(sig2);
        t.alloc.put(sh2);
        t.alloc.put(depth2);
    };
    if (!child2 || !sig2 || !sh2 || !depth2) {
        drop_new();
        return fail(DOT_ENOMEM, "dot_refine: allocation of the refined planes failed");
    }
    if (I > 0)
        hipLaunchKernelGGL(k_child_internal, dim3(blocks_for(I)), dim3(TPB), 0, s, t.child, I, survive, first,
                           rank_int, rank_split, split, cnt_le, nl, child2);
    hipLaunchKernelGGL(k_child_split, dim3(blocks_for(L)), dim3(TPB), 0, s, L, split, rank_split, cnt_le, nl, child2);
    if (t.storage == DOT_F32)
        e = launch_values_emit<DOT_F32>(t, L, I, nv, stride, p.reinit, cover, first, ndepth, need, split, nl, nval, sig2, sh2,
                                        depth2, s);
    else if (t.storage == DOT_F16)
        e = launch_values_emit<DOT_F16>(t, L, I, nv, stride, p.reinit, cover, first, ndepth, need, split, nl, nval, sig2, sh2,
                                        depth2, s);
    else
        e = launch_values_emit<DOT_BF16>(t, L, I, nv, stride, p.reinit, cover, first, ndepth, need, split, nl, nval, sig2, sh2,
                                         depth2, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        drop_new();
        return hip_fail(e, "dot_refine: rebuild");
    }
    // 5. swap into the handle
    t.alloc.put(t.child);
    t.alloc.put(t.sigma);
    t.alloc.put(t.sh);
    t.alloc.put(t.leaf_depth);
    t.child = child2;
    t.sigma = sig2;
    t.sh = sh2;
    t.leaf_depth = depth2;
    t.n_leaves = L2;
    t.n_internal = I2;
    // an upper bound on the deepest leaf (it only bounds traversal steps)
    t.max_depth = std::min(DOT_MAX_DEPTH, t.max_depth + (h_tot[3] > 0 ? 1 : 0));
    if (st_out) {
        st_out->leaves_before = L;
        st_out->leaves_after = L2;
        st_out->internal_after = I2;
        st_out->merged = (int64_t)h_tot[2];
        st_out->subdivided = (int64_t)h_tot[3];
    }
    // the old links described the old topology; without new ones the tree is
    // still complete and walks by re-descent
    return update_links(t, s);
}

}  // namespace dot
