// Face-neighbour links of the leaves (see LINK_* in dot_internal.h), built
// top-down one level per launch.  A node's links are derived from its
// parent's: across a face that stays inside the parent the neighbour is the
// sibling; across a face of the parent the neighbour is the child (mirrored
// octant) of the parent's neighbour when that is an internal node, and the
// parent's neighbour itself, one level further up, when that is a leaf or the
// outside.  The internal nodes of each level are gathered in a frontier list
// for the next launch; leaves write their six links.  Every link is a unique
// value, so the result does not depend on the order of the frontier.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dot_internal.h"

namespace dot {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ uint32_t link_of(int32_t entry, uint32_t up) {
    return entry >= 0 ? (uint32_t)entry : (LINK_LEAF | (up << LINK_ID_BITS) | (uint32_t)(-1 - entry));
}

__global__ void k_links_init(uint32_t* __restrict__ nlinks, int32_t* __restrict__ front, uint32_t* __restrict__ cnt,
                             int n_cnt) {
    const int i = threadIdx.x;
    if (i < 6) nlinks[i] = LINK_OUT;   // the root's faces are the boundary
    if (i == 0) front[0] = 0;
    if (i < n_cnt) cnt[i] = i == 0 ? 1u : 0u;
}

// one thread per (frontier node, octant)
__global__ __launch_bounds__(TPB) void k_links_level(const int32_t* __restrict__ child,
                                                     const uint32_t* __restrict__ cnt_in,
                                                     const int32_t* __restrict__ front_in,
                                                     uint32_t* __restrict__ cnt_out, int32_t* __restrict__ front_out,
                                                     uint32_t* __restrict__ nlinks, uint32_t* __restrict__ links) {
    const int64_t n = (int64_t)(*cnt_in) * 8;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const int64_t node = front_in[i >> 3];
        const int o = (int)(i & 7);
        const int32_t e = child[node * 8 + o];
        uint32_t r[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int a = f >> 1, up = f & 1;
            const int m = o ^ (1 << a);           // octant across the face
            if (((o >> a) & 1) != up) {
                r[f] = link_of(child[node * 8 + m], 0u);   // sibling
            } else {
                const uint32_t q = nlinks[node * 6 + f];
                if (q == LINK_OUT)
                    r[f] = LINK_OUT;
                else if (q & LINK_LEAF)
                    r[f] = q + (1u << LINK_ID_BITS);       // the same leaf, one more level up
                else
                    r[f] = link_of(child[(int64_t)q * 8 + m], 0u);
            }
        }
        uint32_t* dst;
        if (e >= 0) {
            dst = nlinks + (int64_t)e * 6;
            front_out[atomicAdd(cnt_out, 1u)] = e;
        } else {
            dst = links + (int64_t)(-1 - e) * 6;
        }
        uint2* d2 = reinterpret_cast<uint2*>(dst);
        d2[0] = make_uint2(r[0], r[1]);
        d2[1] = make_uint2(r[2], r[3]);
        d2[2] = make_uint2(r[4], r[5]);
    }
}

}  // namespace

int update_links(dot_tree& t, hipStream_t s) {
    t.alloc.put(t.links);
    t.links = nullptr;
    if (!t.links_on || t.n_internal == 0 || t.n_leaves > LINK_MAX_LEAVES) return DOT_OK;
    const int64_t L = t.n_leaves, I = t.n_internal;
    uint32_t* links = static_cast<uint32_t*>(t.alloc.get((size_t)L * 6 * sizeof(uint32_t)));
    // scratch: links of the internal nodes, two frontier lists, one counter per level
    const int n_cnt = DOT_MAX_DEPTH + 1;
    const size_t scratch_bytes = (size_t)I * 6 * 4 + 2 * (size_t)I * 4 + n_cnt * 4;
    char* scratch = static_cast<char*>(t.alloc.get(scratch_bytes));
    if (!links || !scratch) {
        t.alloc.put(links);
        t.alloc.put(scratch);
        return fail(DOT_ENOMEM, "neighbour links: device allocation failed");
    }
    uint32_t* nlinks = reinterpret_cast<uint32_t*>(scratch);
    int32_t* front[2] = {reinterpret_cast<int32_t*>(nlinks + I * 6), reinterpret_cast<int32_t*>(nlinks + I * 6) + I};
    uint32_t* cnt = reinterpret_cast<uint32_t*>(front[1] + I);
    hipLaunchKernelGGL(k_links_init, dim3(1), dim3(64), 0, s, nlinks, front[0], cnt, n_cnt);
    // nodes of depth d (frontier d) place their children; the deepest internal
    // node is at depth max_depth - 1 (max_depth may overstate it)
    const int levels = std::min(std::max(t.max_depth, 1), DOT_MAX_DEPTH);
    const int64_t grid = std::min<int64_t>((I * 8 + TPB - 1) / TPB, 4096);
    for (int d = 0; d < levels; ++d)
        hipLaunchKernelGGL(k_links_level, dim3((unsigned)std::max<int64_t>(grid, 1)), dim3(TPB), 0, s, t.child,
                           cnt + d, front[d & 1], cnt + d + 1, front[(d + 1) & 1], nlinks, links);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    t.alloc.put(scratch);
    if (e != hipSuccess) {
        t.alloc.put(links);
        return hip_fail(e, "neighbour links: build");
    }
    t.links = links;
    return DOT_OK;
}

}  // namespace dot
