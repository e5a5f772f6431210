// Device helpers shared by the render, backward and serving kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dot_internal.h"

namespace dot {

constexpr int WAVE = 64;
constexpr int BLOCK = 128;            // 2 waves, one 8x8 ray tile each
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;

// ---------------------------------------------------------------------------
// Leaf storage: FP32, FP16 or BF16 planes, decoded to FP32 before any math.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ float f16_to_f32(uint32_t h) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

__device__ __forceinline__ uint16_t f32_to_f16(float f) {
    return __builtin_bit_cast(uint16_t, (_Float16)f);  // round to nearest even
}

// round to nearest even on the upper 16 bits; NaN stays NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int DT>
__device__ __forceinline__ float load_sigma(const void* __restrict__ p, int64_t i) {
    if constexpr (DT == DOT_F32) {
        return static_cast<const float*>(p)[i];
    } else {
        uint32_t h = static_cast<const uint16_t*>(p)[i];
        return (DT == DOT_F16 || DT == DOT_PAL16) ? f16_to_f32(h) : bf16_to_f32(h);
    }
}

template <int DT>
constexpr int row_stride(int nv) {
    return DT == DOT_F32 ? (nv + 3) / 4 * 4 : (nv + 7) / 8 * 8;
}

// One leaf's 3K SH coefficients, fetched with 16-byte loads.
template <int DT, int NV>
__device__ __forceinline__ void load_sh_row(const void* __restrict__ base, int64_t leaf, float (&out)[NV]) {
    constexpr int S = row_stride<DT>(NV);
    if constexpr (DT == DOT_F32) {
        const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + leaf * S);
#pragma unroll
        for (int c = 0; c < S / 4; ++c) {
            float4 v = p[c];
            if (4 * c + 0 < NV) out[4 * c + 0] = v.x;
            if (4 * c + 1 < NV) out[4 * c + 1] = v.y;
            if (4 * c + 2 < NV) out[4 * c + 2] = v.z;
            if (4 * c + 3 < NV) out[4 * c + 3] = v.w;
        }
    } else {
        const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + leaf * S);
#pragma unroll
        for (int c = 0; c < S / 8; ++c) {
            uint4 v = p[c];
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                int idx = 8 * c + j;
                if (idx < NV) {
                    uint32_t h = (w[j >> 1] >> ((j & 1) * 16)) & 0xffffu;
                    out[idx] = DT == DOT_F16 ? f16_to_f32(h) : bf16_to_f32(h);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Real orthonormal SH basis, degree <= 3, index k = l^2 + l + m, Condon-Shortley
// phase.  Cartesian forms of sqrt(2) K_l^m P_l^m(cos th) {cos, sin}(m phi) on
// the unit sphere; the constants are sqrt((2l+1)/(4pi) (l-m)!/(l+m)!) times the
// Legendre polynomial factors.
// ---------------------------------------------------------------------------
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float (&Y)[(DEG + 1) * (DEG + 1)]) {
    Y[0] = 0.28209479177387814f;                    // 1/(2 sqrt(pi))
    if constexpr (DEG >= 1) {
        const float c1 = 0.48860251190291992f;      // sqrt(3/(4pi))
        Y[1] = -c1 * y;
        Y[2] = c1 * z;
        Y[3] = -c1 * x;
    }
    if constexpr (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484305920792f * x * y;         // sqrt(15/(4pi))
        Y[5] = -1.0925484305920792f * y * z;
        Y[6] = 0.31539156525252005f * (3.f * zz - 1.f);  // sqrt(5/(16pi))
        Y[7] = -1.0925484305920792f * x * z;
        Y[8] = 0.54627421529603959f * (xx - yy);    // sqrt(15/(16pi))
        if constexpr (DEG >= 3) {
            Y[9] = -0.59004358992664352f * y * (3.f * xx - yy);   // sqrt(35/(32pi))
            Y[10] = 2.8906114426405538f * x * y * z;              // sqrt(105/(4pi))
            Y[11] = -0.45704579946446572f * y * (5.f * zz - 1.f); // sqrt(21/(32pi))
            Y[12] = 0.37317633259011540f * z * (5.f * zz - 3.f);  // sqrt(7/(16pi))
            Y[13] = -0.45704579946446572f * x * (5.f * zz - 1.f);
            Y[14] = 1.4453057213202769f * z * (xx - yy);          // sqrt(105/(16pi))
            Y[15] = -0.59004358992664352f * x * (xx - 3.f * yy);
        }
    }
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sigmoidf_(float x) { return fast_rcp(1.f + __expf(-x)); }

// ---------------------------------------------------------------------------
// Rays
// ---------------------------------------------------------------------------

// Rays are set up in FP64: at a parameter of ~4 an FP32 ray direction or
// crossing time is off by a few 1e-7 world units, and a density jump of 50
// across a leaf boundary turns that into an optical-depth error of ~1e-5.
struct Ray {
    double ox, oy, oz, dx, dy, dz;
};

__device__ __forceinline__ void normalise(Ray& r) {
    double n = 1.0 / sqrt(r.dx * r.dx + r.dy * r.dy + r.dz * r.dz);
    r.dx *= n;
    r.dy *= n;
    r.dz *= n;
}

__device__ __forceinline__ Ray camera_ray(const dot_camera& c, int u, int v) {
    double xc = ((double)u + 0.5 - (double)c.cx) / (double)c.fx;
    double yc = ((double)v + 0.5 - (double)c.cy) / (double)c.fy;
    Ray r;
    r.dx = (double)c.c2w[0] * xc + (double)c.c2w[1] * yc + (double)c.c2w[2];
    r.dy = (double)c.c2w[4] * xc + (double)c.c2w[5] * yc + (double)c.c2w[6];
    r.dz = (double)c.c2w[8] * xc + (double)c.c2w[9] * yc + (double)c.c2w[10];
    r.ox = c.c2w[3];
    r.oy = c.c2w[7];
    r.oz = c.c2w[11];
    normalise(r);
    return r;
}

// Map the wave's tile and lane to a ray.  Returns false for lanes past the
// edge of the image or the end of the ray list.  `rid` = output index.
__device__ __forceinline__ bool make_ray(const RayBatch& rb, int64_t tile, int lane, Ray& r, int64_t& rid) {
    if (rb.kind == DOT_RAYS_CAMERAS) {
        int tw = (rb.width + 7) >> 3, th = (rb.height + 7) >> 3;
        int64_t per = (int64_t)tw * th;
        int cam = (int)(tile / per);
        int t = (int)(tile - (int64_t)cam * per);
        int ty = t / tw, tx = t - ty * tw;
        int u = tx * 8 + (lane & 7), v = ty * 8 + (lane >> 3);
        if (u >= rb.width || v >= rb.height) return false;
        rid = ((int64_t)cam * rb.height + v) * rb.width + u;
        r = camera_ray(rb.cams[cam], u, v);
        return true;
    }
    int64_t i = tile * WAVE + lane;
    if (i >= rb.n_rays) return false;
    rid = i;
    if (rb.kind == DOT_RAYS_PIXELS) {
        const dot_camera& c = rb.cams[rb.cam_idx[i]];
        int p = rb.pix_idx[i];
        int v = p / c.width;
        r = camera_ray(c, p - v * c.width, v);
        return true;
    }
    r.ox = (double)rb.origins[3 * i + 0];
    r.oy = (double)rb.origins[3 * i + 1];
    r.oz = (double)rb.origins[3 * i + 2];
    r.dx = (double)rb.dirs[3 * i + 0];
    r.dy = (double)rb.dirs[3 * i + 1];
    r.dz = (double)rb.dirs[3 * i + 2];
    normalise(r);
    return true;
}

// The ray with output index `rid` of the batch (the index make_ray reports).
__device__ __forceinline__ Ray ray_of(const RayBatch& rb, int64_t rid) {
    Ray r;
    if (rb.kind == DOT_RAYS_CAMERAS) {
        const int64_t hw = (int64_t)rb.width * rb.height;
        const int cam = (int)(rid / hw);
        const int p = (int)(rid - (int64_t)cam * hw);
        const int v = p / rb.width;
        return camera_ray(rb.cams[cam], p - v * rb.width, v);
    }
    if (rb.kind == DOT_RAYS_PIXELS) {
        const dot_camera& c = rb.cams[rb.cam_idx[rid]];
        const int p = rb.pix_idx[rid];
        const int v = p / c.width;
        return camera_ray(c, p - v * c.width, v);
    }
    r.ox = (double)rb.origins[3 * rid + 0];
    r.oy = (double)rb.origins[3 * rid + 1];
    r.oz = (double)rb.origins[3 * rid + 2];
    r.dx = (double)rb.dirs[3 * rid + 0];
    r.dy = (double)rb.dirs[3 * rid + 1];
    r.dz = (double)rb.dirs[3 * rid + 2];
    normalise(r);
    return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD receives a contiguous range of tiles (neighbouring tiles share leaves,
// and each XCD has its own L2).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    int64_t q = nb >> 3, r = nb & 7;
    int64_t x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// ---------------------------------------------------------------------------
// Traversal: walk the leaves along the ray front to back.
//
// Positions live on an integer lattice of 2^LAT cells per axis.  The current
// cell (ix, iy, iz) is the finest cell containing the ray just past the
// current parameter s.  The leaf's exit parameter is the nearest of its three
// exit planes; the axis (or axes, at an edge or corner) that attains it steps
// to the neighbouring cell exactly, and the others take the cell of the exit
// point, clamped to the current leaf's span.  The leaf holding the new cell is
// found
//  - with face-neighbour links (tv.links): when one axis attains the exit,
//    from the link of that face, read together with the leaf's data: a leaf
//    there is the next leaf, an internal node of the same depth is descended
//    by the cell's bits; an exit through an edge or corner descends from the
//    root;
//  - without links: by descending the child array from the deepest ancestor
//    shared with the previous leaf, kept in an LDS stack (one column per lane)
//    and found from the highest differing bit of the old and new cell.
// `seg(leaf, delta)` is called for every segment with delta > 0 and returns
// false to stop the ray.  `desc` counts child-array and link reads.
// ---------------------------------------------------------------------------
template <class Seg>
__device__ __forceinline__ void traverse(const TreeView& tv, const Ray& r, int* __restrict__ stk,
                                         Seg& seg, int& desc) {
    const double LF = (double)LAT_N;
    const double sc = (double)tv.scale;
    double O[3] = {(r.ox - (double)tv.bmin[0]) * sc, (r.oy - (double)tv.bmin[1]) * sc,
                   (r.oz - (double)tv.bmin[2]) * sc};
    double D[3] = {r.dx * sc, r.dy * sc, r.dz * sc};
    double inv[3];
    double t0 = 0.0, t1 = __builtin_huge_val();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (D[a] != 0.0) {
            inv[a] = 1.0 / D[a];
            double p = (0.0 - O[a]) * inv[a], q = (LF - O[a]) * inv[a];
            t0 = fmax(t0, fmin(p, q));
            t1 = fmin(t1, fmax(p, q));
        } else {
            inv[a] = 0.0;
            if (O[a] < 0.0 || O[a] > LF) return;
        }
    }
    if (!(t0 < t1)) return;
    // re-origin at the entry point: positions O + s D for s in [0, t1 - t0]
#pragma unroll
    for (int a = 0; a < 3; ++a) O[a] = fma(t0, D[a], O[a]);
    const double s1 = t1 - t0;
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = min(max((int)floor(O[a]), 0), LAT_N - 1);

    const bool linked = tv.links != nullptr;
    double s = 0.0;
    int nd = 0, k = 0;       // where the next descent starts: node and its depth
    int leaf = -1, ld = 0;   // the leaf holding cell c once known, and its depth
    if (tv.n_internal > 0 && !linked) stk[0] = 0;
    for (int step = 0; step < tv.max_steps; ++step) {
        if (tv.n_internal == 0) {
            leaf = 0;
            ld = 0;
        } else if (leaf < 0) {
            while (true) {
                int sh = LAT - 1 - k;
                int oct = ((c[0] >> sh) & 1) | (((c[1] >> sh) & 1) << 1) | (((c[2] >> sh) & 1) << 2);
                int e = tv.child[(int64_t)nd * 8 + oct];
                ++desc;
                if (e < 0) {
                    leaf = -1 - e;
                    ld = k + 1;
                    break;
                }
                ++k;
                nd = e;
                if (!linked) stk[k * BLOCK] = e;
            }
        }
        const int cs = 1 << (LAT - ld);
        int lo[3];
        double te[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = c[a] & ~(cs - 1);
            if (D[a] > 0.0)
                te[a] = ((double)(lo[a] + cs) - O[a]) * inv[a];
            else if (D[a] < 0.0)
                te[a] = ((double)lo[a] - O[a]) * inv[a];
            else
                te[a] = __builtin_huge_val();
        }
        const double tm = fmin(te[0], fmin(te[1], te[2]));
        const bool last = tm >= s1;
        const double e = fmin(fmax(tm, s), s1);
        const float delta = (float)(e - s);
        // the link across the exit face is requested before the leaf's data so
        // that both arrive in one memory round trip
        const int hits = (te[0] == tm) + (te[1] == tm) + (te[2] == tm);
        uint32_t link = LINK_OUT;
        if (linked && !last && hits == 1) {
            const int ax = te[0] == tm ? 0 : (te[1] == tm ? 1 : 2);
            link = tv.links[(int64_t)leaf * 6 + 2 * ax + (D[ax] > 0.0 ? 1 : 0)];
            ++desc;
        }
        if (delta > 0.f) {
            if (!seg(leaf, delta)) return;
        }
        if (last) return;
        int n[3];
        bool out = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (te[a] == tm) {
                n[a] = D[a] > 0.0 ? lo[a] + cs : lo[a] - 1;
                out |= (unsigned)n[a] >= (unsigned)LAT_N;
            } else {
                int f = (int)floor(fma(tm, D[a], O[a]));
                n[a] = min(max(f, lo[a]), lo[a] + cs - 1);
            }
        }
        if (out) return;
        if (tv.n_internal > 0) {
            if (linked) {
                if (hits != 1) {
                    nd = 0;              // edge or corner: from the root
                    k = 0;
                    leaf = -1;
                } else if (link & LINK_LEAF) {
                    // LINK_OUT is not reached (an interior face has a
                    // neighbour); ids are checked so a bad link cannot
                    // read outside the planes
                    if (link == LINK_OUT || (int64_t)(link & LINK_ID_MASK) >= tv.n_leaves) return;
                    leaf = (int)(link & LINK_ID_MASK);
                    ld -= (int)((link >> LINK_ID_BITS) & 15u);
                } else {
                    if ((int64_t)link >= tv.n_internal) return;
                    nd = (int)link;      // same depth as the leaf just left
                    k = ld;
                    leaf = -1;
                }
            } else {
                unsigned diff = (unsigned)((c[0] ^ n[0]) | (c[1] ^ n[1]) | (c[2] ^ n[2]));
                int cp = __clz(diff) - (32 - LAT);  // depth of the deepest shared ancestor
                k = min(cp, ld - 1);
                nd = stk[k * BLOCK];
                leaf = -1;
            }
        }
        c[0] = n[0];
        c[1] = n[1];
        c[2] = n[2];
        s = e;
    }
}

// Per-ray compositing state for the forward pass.  S is the optical depth so
// far (log of the transmittance, kept in FP32), T = exp(-S).  A segment's
// weight is w = T_i - T_{i+1} = T_i (1 - exp(-tau_i)).
template <int DT, int DEG, bool COUNT = false>
struct FwdSeg {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    const TreeView& tv;
    const FwdArgs& a;
    float Y[K];
    float S = 0.f, T = 1.f;
    float C[3] = {0.f, 0.f, 0.f};
    int n = 0;
    int fetched = 0;
    int64_t rid = 0;    // COUNT: the ray's index in the batch (record column)
    int nrec = 0;       // COUNT: composited segments recorded so far
    // COUNT: the last record's bucket slot is stored with the next record (or
    // at the end of the ray), so the forward never waits for the atomic
    int64_t pend_j = -1;
    uint32_t pend_slot = 0;

    __device__ FwdSeg(const TreeView& tv_, const FwdArgs& a_) : tv(tv_), a(a_) {}

    __device__ __forceinline__ void flush_slot() {
        if constexpr (COUNT)
            if (pend_j >= 0) a.rec.slot[pend_j] = pend_slot;
    }

    __device__ __forceinline__ bool operator()(int leaf, float delta) {
        // sigma and the SH row are requested together (one memory round trip);
        // a leaf with sigma^ delta = 0 contributes w = 0
        float sg = fmaxf(load_sigma<DT>(tv.sigma, leaf), 0.f);
        // the stored signal, read for the max filter below, is requested with the
        // leaf data so it does not add a dependent load after compositing
        const float cur = a.signal ? a.signal[leaf] : 0.f;
        // BF16 rows stay packed in registers and each coefficient is widened in
        // the dot product (FP16 rows stay packed through mixed-precision FMAs)
        constexpr int NW = (3 * K + 1) / 2;
        float row[DT == DOT_BF16 ? 1 : 3 * K];
        uint32_t packed[DT == DOT_BF16 ? NW : 1];
        if constexpr (DT == DOT_BF16) {
            const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(tv.sh) + (int64_t)leaf * row_stride<DT>(3 * K));
#pragma unroll
            for (int c = 0; c < (NW + 3) / 4; ++c) {
                uint4 v = p[c];
                if (4 * c + 0 < NW) packed[4 * c + 0] = v.x;
                if (4 * c + 1 < NW) packed[4 * c + 1] = v.y;
                if (4 * c + 2 < NW) packed[4 * c + 2] = v.z;
                if (4 * c + 3 < NW) packed[4 * c + 3] = v.w;
            }
        } else if constexpr (DT == DOT_PAL16) {
            // the row lives in the palette: one dependent load after the index
            const uint32_t pi = static_cast<const uint16_t*>(tv.sh)[leaf];
            load_sh_row<DOT_F16, 3 * K>(tv.palette, pi, row);
        } else {
            load_sh_row<DT, 3 * K>(tv.sh, leaf, row);
        }
        float tau = sg * delta;
        ++n;
        fetched += tau > 0.f;
        // a training forward counts, per leaf, the segments whose gradient rows
        // its adjoint emits; a segment it records also reserves its row's slot
        // in the leaf's bucket (issued here, early, and consumed one record later)
        [[maybe_unused]] uint32_t slot = 0;
        [[maybe_unused]] bool record = false;
        if constexpr (COUNT) {
            if (sg > 0.f) {
                if (a.rec.a && nrec < a.rec.cap) {
                    slot = atomicAdd(&a.leaf_count[leaf], 1u);
                    record = true;
                } else {
                    atomicAdd(&a.leaf_rest[leaf], 1u);
                }
            }
        }
        {
            float Sn = S + tau;
            float Tn = __expf(-Sn);
            float w = fmaxf(T - Tn, 0.f);
            float cv[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float x = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    float cf;
                    if constexpr (DT == DOT_BF16) {
                        int i = ch * K + k;
                        uint32_t wv = packed[i >> 1];
                        cf = __uint_as_float((i & 1) ? (wv & 0xffff0000u) : (wv << 16));
                    } else {
                        cf = row[ch * K + k];
                    }
                    x = fmaf(cf, Y[k], x);
                }
                cv[ch] = sigmoidf_(x);
                C[ch] = fmaf(w, cv[ch], C[ch]);
            }
            // the record the adjoint replays: leaf, delta, tau, the colour and
            // (stored with the next record) the reserved slot
            if constexpr (COUNT) {
                if (record) {
                    const int64_t j = (int64_t)nrec * a.rec.n + rid;
                    a.rec.a[j] = make_float4(__int_as_float(leaf), delta, tau, cv[0]);
                    a.rec.b[j] = make_float2(cv[1], cv[2]);
                    flush_slot();
                    pend_j = j;
                    pend_slot = slot;
                }
                if (sg > 0.f && a.rec.a) ++nrec;
            }
            if (a.signal) {
                if (a.signal_mode == DOT_SIGNAL_MAX) {
                    // non-negative floats order like their bit patterns; skip the
                    // atomic when the stored value already dominates
                    if (w > cur) atomicMax(reinterpret_cast<unsigned int*>(&a.signal[leaf]), __float_as_uint(w));
                } else {
                    unsafeAtomicAdd(&a.signal[leaf], w);
                }
            }
            S = Sn;
            T = Tn;
        }
        return !(S > a.thr);
    }
};

}  // namespace dot
