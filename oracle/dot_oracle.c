/*
 * FP64 CPU oracle for the Dynamic PlenOctree (DOT) octree volume renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * it is used by the test suite, by the smoke check and by the benchmark's CPU
 * baseline.  It shares no code, header or constant with the HIP library; the
 * two meet only in the canonical input arrays.
 *
 * What it computes, and from which passage of the paper:
 *
 *  - Rendering, Sec. 3 "Preliminaries", Eq. 1-2: a ray crosses the leaves of
 *    the octree, each with constant density sigma_i and SH colour c_i, over
 *    segments delta_i.  C = sum_i T_i Q_i c_i with Q_i = 1 - exp(-sigma_i
 *    delta_i) and T_i = exp(-sum_{j<i} sigma_j delta_j); the remaining
 *    transmittance multiplies a background colour.  For a piecewise-constant
 *    field this sum IS the emission-absorption integral, so the oracle is the
 *    definition written out: the ordered segments are found by a recursive
 *    front-to-back descent that clips the ray interval against each child
 *    box (a different algorithm from the GPU's lattice stepping).
 *  - Colour c_i "in the form of SH" (Sec. 3): real orthonormal spherical
 *    harmonics evaluated from the associated-Legendre definition with the
 *    Condon-Shortley phase, followed by a sigmoid (or the identity, used only
 *    by closed-form checks).
 *  - Training signal Q (Sec. 3.1, Alg. 1 render returns Q): per leaf, the max
 *    (default) or the sum over rays of the ray weight w_i = T_i Q_i.
 *  - Gradient of the MSE objective (Sec. 3 Preliminaries, the renderer is
 *    fully differentiable): analytic adjoint of Eq. 1-2 in FP64.
 *  - Refinement (Sec. 3.2, Eq. 3 pruning = mean of the M=8 children, Eq. 4
 *    sampling = copy a leaf into 8 children; selection {Q <= tau} and
 *    topk(gamma, Q) of Alg. 1), written as a recursive rebuild of the tree.
 *
 * Readings where the paper is silent are stated at each function.
 * Early termination: a ray stops after the segment that drives exp(-S) below
 * t_stop.  Because FP32 and FP64 can take that decision differently when S is
 * within rounding of -ln(t_stop), the oracle also reports the results of the
 * stopping rule moved by +-margin in S ("early" and "late" branches).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

typedef struct {
    int64_t n_internal;
    int64_t n_leaves;
    int32_t degree;
    int32_t sh_f64;        /* 1: sh points to doubles, 0: to floats        */
    const int32_t *child;  /* [n_internal][8]; >=0 internal, <0 leaf -1-id */
    const double *sigma;   /* [L]      raw stored density (upcast)        */
    const void *sh;        /* [L][3][K] raw stored coefficients (upcast)   */
    double bmin[3];
    double size;
} orc_tree;

typedef struct {
    float c2w[12];
    float fx, fy, cx, cy;
    int32_t width, height;
} orc_camera;

typedef struct {
    double bg[3];
    double t_stop;     /* 0 disables early termination */
    double margin;     /* straddle window on S for the early/late branches */
    int32_t activation; /* 0 sigmoid, 1 identity */
    int32_t signal_mode; /* 0 max over rays, 1 sum over rays */
} orc_opts;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3 (index k = l^2 + l + m).            */
/*   Y_l^0      = K_l^0 P_l^0(cos th)                                       */
/*   Y_l^{+m}   = sqrt(2) K_l^m P_l^m(cos th) cos(m phi)                     */
/*   Y_l^{-m}   = sqrt(2) K_l^m P_l^m(cos th) sin(m phi)                     */
/*   K_l^m      = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)                         */
/* P_l^m carries the Condon-Shortley phase (-1)^m.                           */
/* ------------------------------------------------------------------------ */

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* associated Legendre P_l^m(x), m >= 0, by the standard three-term recurrence */
static double assoc_legendre(int l, int m, double x) {
    double pmm = 1.0;
    double s = sqrt((1.0 - x) * (1.0 + x));
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s; /* (-1)^m (2m-1)!! s^m */
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pll;
    }
    return pll;
}

void orc_sh_basis(int degree, const double dir[3], double *out) {
    double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double x = dir[0] / n, y = dir[1] / n, z = dir[2] / n;
    double phi = atan2(y, x);
    for (int l = 0; l <= degree; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * factorial(l - am) / factorial(l + am));
            double P = assoc_legendre(l, am, z);
            double v;
            if (m == 0)
                v = K * P;
            else if (m > 0)
                v = sqrt(2.0) * K * P * cos(m * phi);
            else
                v = sqrt(2.0) * K * P * sin(am * phi);
            out[l * l + l + m] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pinhole rays: o = camera centre; d = normalize(R ((u+.5-cx)/fx,          */
/* (v+.5-cy)/fy, 1)); camera x right, y down, z forward; pixel p = v W + u.  */
/* ------------------------------------------------------------------------ */

void orc_camera_rays(const orc_camera *cams, int64_t n, const int32_t *cam_idx,
                     const int32_t *pix_idx, double *o, double *d) {
    for (int64_t r = 0; r < n; ++r) {
        const orc_camera *c = &cams[cam_idx[r]];
        int64_t p = pix_idx[r];
        double u = (double)(p % c->width), v = (double)(p / c->width);
        double cx = ((u + 0.5) - (double)c->cx) / (double)c->fx;
        double cy = ((v + 0.5) - (double)c->cy) / (double)c->fy;
        double dw[3];
        for (int a = 0; a < 3; ++a)
            dw[a] = (double)c->c2w[4 * a + 0] * cx + (double)c->c2w[4 * a + 1] * cy +
                    (double)c->c2w[4 * a + 2];
        double nn = sqrt(dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2]);
        for (int a = 0; a < 3; ++a) {
            o[3 * r + a] = (double)c->c2w[4 * a + 3];
            d[3 * r + a] = dw[a] / nn;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Ordered leaf segments of one ray                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t *leaf;
    double *delta;
    int64_t n, cap;
} seglist;

static void seg_push(seglist *s, int32_t leaf, double delta) {
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 64;
        s->leaf = (int32_t *)realloc(s->leaf, sizeof(int32_t) * s->cap);
        s->delta = (double *)realloc(s->delta, sizeof(double) * s->cap);
    }
    s->leaf[s->n] = leaf;
    s->delta[s->n] = delta;
    s->n++;
}

/* Interval of t for which o + t d lies in the box [lo, lo+size]^3, intersected
 * with [ta, tb].  Returns 0 if empty (a >= b).  Leaves tile the root, so every
 * point belongs to exactly one cell: cells are half-open, [lo, lo+size) per
 * axis, except that the root's upper faces belong to the last cell.  This
 * matters only for a ray that lies in a cell plane (d[k] == 0); for any other
 * ray the half-open and closed boxes give the same interval. */
static int clip_box(const orc_tree *T, const double lo[3], double size, const double o[3], const double d[3],
                    double ta, double tb, double *a_out, double *b_out) {
    double a = ta, b = tb;
    for (int k = 0; k < 3; ++k) {
        double p0 = lo[k], p1 = lo[k] + size;
        if (d[k] == 0.0) {
            int top = (p1 == T->bmin[k] + T->size);
            if (o[k] < p0 || o[k] > p1 || (o[k] == p1 && !top)) return 0;
            continue;
        }
        double t0 = (p0 - o[k]) / d[k];
        double t1 = (p1 - o[k]) / d[k];
        if (t0 > t1) { double tmp = t0; t0 = t1; t1 = tmp; }
        if (t0 > a) a = t0;
        if (t1 < b) b = t1;
    }
    *a_out = a;
    *b_out = b;
    return a < b;
}

static void descend(const orc_tree *T, int32_t entry, const double lo[3], double size,
                    const double o[3], const double d[3], double ta, double tb, seglist *out) {
    if (entry < 0) {
        double delta = tb - ta;
        if (delta > 0.0) seg_push(out, -1 - entry, delta);
        return;
    }
    double half = 0.5 * size;
    double ca[8], cb[8];
    int order[8], nk = 0;
    for (int oc = 0; oc < 8; ++oc) {
        double clo[3] = {lo[0] + ((oc & 1) ? half : 0.0), lo[1] + ((oc & 2) ? half : 0.0),
                         lo[2] + ((oc & 4) ? half : 0.0)};
        double a, b;
        if (clip_box(T, clo, half, o, d, ta, tb, &a, &b)) {
            ca[oc] = a;
            cb[oc] = b;
            /* insertion sort by entry t; equal entries keep octant order */
            int j = nk++;
            while (j > 0 && ca[order[j - 1]] > a) {
                order[j] = order[j - 1];
                --j;
            }
            order[j] = oc;
        }
    }
    for (int j = 0; j < nk; ++j) {
        int oc = order[j];
        double clo[3] = {lo[0] + ((oc & 1) ? half : 0.0), lo[1] + ((oc & 2) ? half : 0.0),
                         lo[2] + ((oc & 4) ? half : 0.0)};
        descend(T, T->child[8 * (int64_t)entry + oc], clo, half, o, d, ca[oc], cb[oc], out);
    }
}

static void ray_segments(const orc_tree *T, const double o[3], const double d_in[3], seglist *out) {
    double n = sqrt(d_in[0] * d_in[0] + d_in[1] * d_in[1] + d_in[2] * d_in[2]);
    double d[3] = {d_in[0] / n, d_in[1] / n, d_in[2] / n};
    double a, b;
    out->n = 0;
    if (!clip_box(T, T->bmin, T->size, o, d, 0.0, INFINITY, &a, &b)) return;
    int32_t root = T->n_internal > 0 ? 0 : -1; /* a root that is a leaf is leaf 0 */
    descend(T, root, T->bmin, T->size, o, d, a, b, out);
}

/* Public: segments of one ray (for tests).  Returns the total count; writes at most cap. */
int64_t orc_ray_segments(const orc_tree *T, const double o[3], const double d[3],
                         int32_t *leaf, double *delta, int64_t cap) {
    seglist s = {0, 0, 0, 0};
    ray_segments(T, o, d, &s);
    for (int64_t i = 0; i < s.n && i < cap; ++i) {
        leaf[i] = s.leaf[i];
        delta[i] = s.delta[i];
    }
    int64_t n = s.n;
    free(s.leaf);
    free(s.delta);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Compositing                                                               */
/* ------------------------------------------------------------------------ */

static int sh_count(int degree) { return (degree + 1) * (degree + 1); }

static double sh_at(const orc_tree *T, int64_t j) {
    return T->sh_f64 ? ((const double *)T->sh)[j] : (double)((const float *)T->sh)[j];
}

static double activate(int act, double x) { return act == 1 ? x : 1.0 / (1.0 + exp(-x)); }
static double activate_grad(int act, double c) { return act == 1 ? 1.0 : c * (1.0 - c); }

/* colour of leaf `l` for basis Y */
static void leaf_colour(const orc_tree *T, int64_t l, const double *Y, int act, double c[3]) {
    int K = sh_count(T->degree);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += sh_at(T, (l * 3 + ch) * K + k) * Y[k];
        c[ch] = activate(act, acc);
    }
}

/* per-segment record kept for the signal: weight and which branches include it */
typedef struct {
    int32_t leaf;
    uint8_t in_early, in_primary;
    double w;
} sigrec;

/* Composite one ray.  Variants: 0 = early (threshold - margin), 1 = primary,
 * 2 = late (threshold + margin).  A variant "stops" after the first segment
 * whose running optical depth S exceeds its threshold. */
static void composite(const orc_tree *T, const seglist *s, const double *Y, const orc_opts *opt,
                      double rgb[3][3], int32_t nseg[3], sigrec *rec) {
    double thr = opt->t_stop > 0.0 ? -log(opt->t_stop) : INFINITY;
    double lim[3] = {thr - opt->margin, thr, thr + opt->margin};
    int done[3] = {0, 0, 0};
    double S = 0.0, C[3] = {0, 0, 0};
    int64_t i;
    for (i = 0; i < s->n; ++i) {
        int32_t l = s->leaf[i];
        double sg = T->sigma[l] > 0.0 ? T->sigma[l] : 0.0; /* density activation: ReLU */
        double tau = sg * s->delta[i];
        double alpha = -expm1(-tau);
        double w = exp(-S) * alpha;
        double c[3];
        leaf_colour(T, l, Y, opt->activation, c);
        for (int ch = 0; ch < 3; ++ch) C[ch] += w * c[ch];
        rec[i].leaf = l;
        rec[i].w = w;
        rec[i].in_early = !done[0];
        rec[i].in_primary = !done[1];
        S += tau;
        for (int v = 0; v < 3; ++v) {
            if (!done[v] && S > lim[v]) {
                done[v] = 1;
                double Tn = exp(-S);
                for (int ch = 0; ch < 3; ++ch) rgb[v][ch] = C[ch] + Tn * opt->bg[ch];
                nseg[v] = (int32_t)(i + 1);
            }
        }
        if (done[2]) { ++i; break; }
    }
    double Tn = exp(-S);
    for (int v = 0; v < 3; ++v) {
        if (!done[v]) {
            for (int ch = 0; ch < 3; ++ch) rgb[v][ch] = C[ch] + Tn * opt->bg[ch];
            nseg[v] = (int32_t)i;
        }
    }
    /* records past the late stop do not exist (loop broke) */
    for (int64_t j = i; j < s->n; ++j) rec[j].leaf = -1;
}

/*
 * Render n rays.  Outputs (any may be NULL):
 *   rgb, rgb_early, rgb_late  [n][3]
 *   nseg                      [n]  segments composited by the primary rule
 *   flags                     [n]  bit0: early and late branches differ
 *   sig, sig_lo, sig_hi       [L]  signal under the primary / early / late rule
 *                                  (accumulated into: max or +=)
 */
void orc_render(const orc_tree *T, int64_t n, const double *o, const double *d, const orc_opts *opt,
                double *rgb, double *rgb_early, double *rgb_late, int32_t *nseg, int32_t *flags,
                double *sig, double *sig_lo, double *sig_hi) {
    int K = sh_count(T->degree);
    int want_sig = sig || sig_lo || sig_hi;
    sigrec **recs = want_sig ? (sigrec **)calloc((size_t)n, sizeof(sigrec *)) : NULL;
    int64_t *nrec = want_sig ? (int64_t *)calloc((size_t)n, sizeof(int64_t)) : NULL;
#pragma omp parallel
    {
        seglist s = {0, 0, 0, 0};
        sigrec *rec = NULL;
        int64_t rcap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n; ++r) {
            ray_segments(T, &o[3 * r], &d[3 * r], &s);
            double Y[16];
            orc_sh_basis(T->degree, &d[3 * r], Y);
            (void)K;
            if (s.n > rcap) {
                rcap = s.n;
                rec = (sigrec *)realloc(rec, sizeof(sigrec) * rcap);
            }
            double out[3][3];
            int32_t ns[3];
            composite(T, &s, Y, opt, out, ns, rec);
            for (int ch = 0; ch < 3; ++ch) {
                if (rgb) rgb[3 * r + ch] = out[1][ch];
                if (rgb_early) rgb_early[3 * r + ch] = out[0][ch];
                if (rgb_late) rgb_late[3 * r + ch] = out[2][ch];
            }
            if (nseg) nseg[r] = ns[1];
            if (flags) flags[r] = (ns[0] != ns[2]) ? 1 : 0;
            if (want_sig) {
                int64_t m = 0;
                for (int64_t i = 0; i < s.n; ++i)
                    if (rec[i].leaf >= 0) ++m;
                recs[r] = (sigrec *)malloc(sizeof(sigrec) * (m ? m : 1));
                memcpy(recs[r], rec, sizeof(sigrec) * m);
                nrec[r] = m;
            }
        }
        free(s.leaf);
        free(s.delta);
        free(rec);
    }
    if (want_sig) {
        /* serial reduction in ray order (deterministic) */
        for (int64_t r = 0; r < n; ++r) {
            for (int64_t i = 0; i < nrec[r]; ++i) {
                const sigrec *q = &recs[r][i];
                double w = q->w;
                if (opt->signal_mode == 0) {
                    if (sig_hi && w > sig_hi[q->leaf]) sig_hi[q->leaf] = w;
                    if (sig && q->in_primary && w > sig[q->leaf]) sig[q->leaf] = w;
                    if (sig_lo && q->in_early && w > sig_lo[q->leaf]) sig_lo[q->leaf] = w;
                } else {
                    if (sig_hi) sig_hi[q->leaf] += w;
                    if (sig && q->in_primary) sig[q->leaf] += w;
                    if (sig_lo && q->in_early) sig_lo[q->leaf] += w;
                }
            }
            free(recs[r]);
        }
        free(recs);
        free(nrec);
    }
}

/* ------------------------------------------------------------------------ */
/* Analytic gradient (primary stopping rule).                                */
/*   dC/dtau_i = T_{i+1} c_i - (C - P_i),  P_i = sum_{j<=i} w_j c_j,         */
/*   where C includes the background term; dtau_i/dsigma_i = delta_i for     */
/*   sigma_i > 0 and 0 otherwise (ReLU, subgradient 0 at 0);                 */
/*   dC_ch/dsh[ch][k] = w_i act'(c) Y_k.                                     */
/* grad_sigma [L] and grad_sh [L][3][K] are accumulated into (+=).           */
/* ------------------------------------------------------------------------ */
void orc_backward(const orc_tree *T, int64_t n, const double *o, const double *d, const orc_opts *opt,
                  const double *grad_rgb, double *grad_sigma, double *grad_sh) {
    int K = sh_count(T->degree);
    int64_t L = T->n_leaves;
    int64_t P = L * (1 + 3 * K);
    int nt = orc_num_threads();
    /* per-thread accumulators when they fit, else serial */
    if ((double)P * nt * 8.0 > 4e9) nt = 1;
    double *acc = (double *)calloc((size_t)P * nt, sizeof(double));
    double thr = opt->t_stop > 0.0 ? -log(opt->t_stop) : INFINITY;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gs = acc + (size_t)P * tid;
        double *gh = gs + L;
        seglist s = {0, 0, 0, 0};
        double *cc = NULL, *ww = NULL, *tn = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n; ++r) {
            ray_segments(T, &o[3 * r], &d[3 * r], &s);
            double Y[16];
            orc_sh_basis(T->degree, &d[3 * r], Y);
            if (s.n > cap) {
                cap = s.n;
                cc = (double *)realloc(cc, sizeof(double) * 3 * cap);
                ww = (double *)realloc(ww, sizeof(double) * cap);
                tn = (double *)realloc(tn, sizeof(double) * cap);
            }
            /* forward */
            double S = 0.0, C[3] = {0, 0, 0};
            int64_t m = 0;
            for (int64_t i = 0; i < s.n; ++i) {
                int32_t l = s.leaf[i];
                double sg = T->sigma[l] > 0.0 ? T->sigma[l] : 0.0;
                double tau = sg * s.delta[i];
                double Ti = exp(-S);
                double w = Ti * (-expm1(-tau));
                leaf_colour(T, l, Y, opt->activation, &cc[3 * i]);
                for (int ch = 0; ch < 3; ++ch) C[ch] += w * cc[3 * i + ch];
                S += tau;
                ww[i] = w;
                tn[i] = exp(-S);
                m = i + 1;
                if (S > thr) break;
            }
            double Tend = exp(-S);
            for (int ch = 0; ch < 3; ++ch) C[ch] += Tend * opt->bg[ch];
            /* adjoint */
            const double *g = &grad_rgb[3 * r];
            double Pc[3] = {0, 0, 0};
            for (int64_t i = 0; i < m; ++i) {
                int32_t l = s.leaf[i];
                const double *c = &cc[3 * i];
                for (int ch = 0; ch < 3; ++ch) Pc[ch] += ww[i] * c[ch];
                if (T->sigma[l] > 0.0) {
                    double dt = 0.0;
                    for (int ch = 0; ch < 3; ++ch) dt += g[ch] * (tn[i] * c[ch] - (C[ch] - Pc[ch]));
                    gs[l] += dt * s.delta[i];
                }
                for (int ch = 0; ch < 3; ++ch) {
                    double f = g[ch] * ww[i] * activate_grad(opt->activation, c[ch]);
                    for (int k = 0; k < K; ++k) gh[(l * 3 + ch) * K + k] += f * Y[k];
                }
            }
        }
        free(s.leaf);
        free(s.delta);
        free(cc);
        free(ww);
        free(tn);
    }
    for (int t = 0; t < nt; ++t) {
        const double *gs = acc + (size_t)P * t;
        for (int64_t l = 0; l < L; ++l) grad_sigma[l] += gs[l];
        for (int64_t j = 0; j < 3 * K * L; ++j) grad_sh[j] += gs[L + j];
    }
    free(acc);
}

/* ------------------------------------------------------------------------ */
/* Rounding to the leaf storage formats, from the IEEE-754 definition:       */
/* round to nearest, ties to even, at p significant bits; below the minimum  */
/* normal exponent the quantum is fixed (gradual underflow); beyond the      */
/* largest finite value the result is infinite.                              */
/* storage: 0 FP32, 1 FP16, 2 BF16                                           */
/* ------------------------------------------------------------------------ */
double orc_round_storage(int storage, double x) {
    int p, emin;
    double maxf;
    if (storage == 1) { p = 11; emin = -14; maxf = 65504.0; }
    else if (storage == 2) { p = 8; emin = -126; maxf = 3.38953138925153547590e38; }
    else { p = 24; emin = -126; maxf = 3.40282346638528859812e38; }
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);        /* |x| in [2^(e-1), 2^e) */
    int lead = e - 1;
    if (lead < emin) lead = emin;
    double q = ldexp(1.0, lead - (p - 1));
    double r = nearbyint(x / q) * q; /* default rounding mode: nearest-even */
    if (fabs(r) > maxf) return x > 0 ? INFINITY : -INFINITY;
    return r;
}

void orc_round_storage_array(int storage, int64_t n, const double *in, double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = orc_round_storage(storage, in[i]);
}

/* ------------------------------------------------------------------------ */
/* Refinement (Sec. 3.2, Alg. 1 pruning then sampling from the same signal) */
/*  - prune selection: s <= tau (prune_le = 1) or s < tau (prune_le = 0)     */
/*  - an internal node merges iff all 8 children are leaves and selected;   */
/*    the new leaf holds the FP64 mean of the children's raw sigma and SH   */
/*    (Eq. 3, M = 8), rounded once to the storage format                    */
/*  - sampling candidates: leaves not selected for pruning with depth <     */
/*    max_depth; the first k = floor(sample_frac * L) of them by (signal    */
/*    descending, DFS index ascending) are split into 8 children holding    */
/*    copies of the parent's values (Eq. 4)                                 */
/*  - recursive (the paper's "(R)" option): merging repeats on the merged   */
/*    tree, a merged node's signal being the max of its children's, until  */
/*    no group is selected; sampling then uses the original leaves' signal  */
/*  The new tree is numbered in DFS order.                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double tau;
    double sample_frac;
    int32_t prune_le;
    int32_t max_depth;
    int32_t recursive;
    int32_t storage;
    int32_t reinit;    /* 1: new leaves start from zero instead of the fused values */
    int32_t pad_;
} orc_refine_params;

typedef struct {
    int64_t n_internal, n_leaves, merged, subdivided, k;
    int32_t *child;
    double *sigma;
    float *sh;
    int32_t *depth;
    uint64_t *morton; /* Morton code of the leaf cell at its own depth */
} orc_refined;

typedef struct {
    const orc_tree *T;
    const orc_refine_params *P;
    int K;
    /* per old internal node */
    int32_t *node_depth;
    uint8_t *merge;      /* node becomes a leaf */
    double *node_sig;    /* signal of a merged node (recursive mode) */
    /* per old leaf */
    int32_t *leaf_depth;
    uint8_t *split;
    const float *signal;
    orc_refined *out;
    int64_t cap_int, cap_leaf;
} rf_ctx;

static void rf_depths(rf_ctx *c, int32_t node, int32_t depth) {
    c->node_depth[node] = depth;
    for (int oc = 0; oc < 8; ++oc) {
        int32_t e = c->T->child[8 * (int64_t)node + oc];
        if (e >= 0) rf_depths(c, e, depth + 1);
        else c->leaf_depth[-1 - e] = depth + 1;
    }
}

static int rf_selected(const rf_ctx *c, double s) {
    return c->P->prune_le ? (s <= c->P->tau) : (s < c->P->tau);
}

/* one merge pass over nodes whose children are all leaves-or-merged;
 * returns the number of new merges */
static int64_t rf_merge_pass(rf_ctx *c, int first_pass) {
    int64_t added = 0;
    /* children have larger indices than parents in pre-order: scan backwards */
    for (int64_t p = c->T->n_internal - 1; p >= 0; --p) {
        if (c->merge[p]) continue;
        int all = 1;
        double mx = 0.0;
        for (int oc = 0; oc < 8 && all; ++oc) {
            int32_t e = c->T->child[8 * p + oc];
            double s;
            if (e < 0) s = (double)c->signal[-1 - e];
            else if (!first_pass && c->merge[e]) s = c->node_sig[e];
            else { all = 0; break; }
            if (!rf_selected(c, s)) all = 0;
            if (s > mx) mx = s;
        }
        if (all) {
            c->merge[p] = 2; /* merged in this pass */
            c->node_sig[p] = mx;
            ++added;
        }
    }
    for (int64_t p = 0; p < c->T->n_internal; ++p)
        if (c->merge[p] == 2) c->merge[p] = 1;
    return added;
}

/* `fresh` marks a leaf created by this refinement (a merged node or a child of
 * a subdivided leaf); with reinit such leaves start from zero -- the paper's
 * ablation that disables feature fusion (App. C.1) -- instead of Eq. 3 / Eq. 4 */
static void rf_push_leaf(rf_ctx *c, int32_t depth, uint64_t morton, const double *sig, const double *sh,
                         int fresh) {
    orc_refined *o = c->out;
    int64_t l = o->n_leaves++;
    int K = c->K;
    int zero = fresh && c->P->reinit;
    o->depth[l] = depth;
    o->morton[l] = morton;
    o->sigma[l] = zero ? 0.0 : orc_round_storage(c->P->storage, sig[0]);
    for (int j = 0; j < 3 * K; ++j) o->sh[l * 3 * K + j] = zero ? 0.0f : (float)orc_round_storage(c->P->storage, sh[j]);
}

/* mean of the stored values of all leaves under `node` when the subtree is
 * merged; for a one-level merge this is Eq. 3 over the 8 children.  A
 * recursive merge averages the averages of its children (each rounded to
 * storage when it was formed), following Eq. 3 applied level by level. */
static void rf_subtree_value(rf_ctx *c, int32_t entry, double *sig, double *sh) {
    int K = c->K;
    if (entry < 0) {
        int64_t l = -1 - entry;
        sig[0] = c->T->sigma[l];
        for (int j = 0; j < 3 * K; ++j) sh[j] = sh_at(c->T, l * 3 * K + j);
        return;
    }
    double cs[8], csh[8][48];
    for (int oc = 0; oc < 8; ++oc) rf_subtree_value(c, c->T->child[8 * (int64_t)entry + oc], &cs[oc], csh[oc]);
    double acc = 0.0;
    for (int oc = 0; oc < 8; ++oc) acc += cs[oc];
    sig[0] = orc_round_storage(c->P->storage, acc / 8.0);
    for (int j = 0; j < 3 * K; ++j) {
        double a = 0.0;
        for (int oc = 0; oc < 8; ++oc) a += csh[oc][j];
        sh[j] = orc_round_storage(c->P->storage, a / 8.0);
    }
}

static uint64_t rf_child_morton(uint64_t m, int oc) { return (m << 3) | (uint64_t)oc; }

/* rebuild; returns the new child-array entry for this subtree */
static int32_t rf_build(rf_ctx *c, int32_t entry, int32_t depth, uint64_t morton) {
    orc_refined *o = c->out;
    int K = c->K;
    double sig, sh[48];
    if (entry >= 0 && !c->merge[entry]) {
        int64_t me = o->n_internal++;
        for (int oc = 0; oc < 8; ++oc) {
            int32_t v = rf_build(c, c->T->child[8 * (int64_t)entry + oc], depth + 1, rf_child_morton(morton, oc));
            o->child[8 * me + oc] = v;
        }
        return (int32_t)me;
    }
    if (entry >= 0) { /* merged node -> one leaf */
        rf_subtree_value(c, entry, &sig, sh);
        int64_t l = o->n_leaves;
        rf_push_leaf(c, depth, morton, &sig, sh, 1);
        return (int32_t)(-1 - l);
    }
    int64_t old = -1 - entry;
    sig = c->T->sigma[old];
    for (int j = 0; j < 3 * K; ++j) sh[j] = sh_at(c->T, old * 3 * K + j);
    if (c->split[old]) {
        int64_t me = o->n_internal++;
        for (int oc = 0; oc < 8; ++oc) {
            int64_t l = o->n_leaves;
            rf_push_leaf(c, depth + 1, rf_child_morton(morton, oc), &sig, sh, 1);
            o->child[8 * me + oc] = (int32_t)(-1 - l);
        }
        return (int32_t)me;
    }
    int64_t l = o->n_leaves;
    rf_push_leaf(c, depth, morton, &sig, sh, 0);
    return (int32_t)(-1 - l);
}

typedef struct {
    double s;
    int64_t idx;
} rf_key;

static int rf_cmp(const void *a, const void *b) {
    const rf_key *x = (const rf_key *)a, *y = (const rf_key *)b;
    if (x->s > y->s) return -1;
    if (x->s < y->s) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

void orc_refined_free(orc_refined *r) {
    free(r->child);
    free(r->sigma);
    free(r->sh);
    free(r->depth);
    free(r->morton);
    memset(r, 0, sizeof(*r));
}

int orc_refine(const orc_tree *T, const float *signal, const orc_refine_params *P, orc_refined *out) {
    rf_ctx c;
    memset(&c, 0, sizeof(c));
    memset(out, 0, sizeof(*out));
    c.T = T;
    c.P = P;
    c.K = sh_count(T->degree);
    c.signal = signal;
    c.out = out;
    int64_t I = T->n_internal, L = T->n_leaves;
    c.node_depth = (int32_t *)calloc(I ? I : 1, sizeof(int32_t));
    c.merge = (uint8_t *)calloc(I ? I : 1, 1);
    c.node_sig = (double *)calloc(I ? I : 1, sizeof(double));
    c.leaf_depth = (int32_t *)calloc(L, sizeof(int32_t));
    c.split = (uint8_t *)calloc(L, 1);
    if (I > 0) rf_depths(&c, 0, 0);
    else c.leaf_depth[0] = 0;
    /* pruning */
    int64_t merged = 0;
    if (I > 0) {
        int64_t a = rf_merge_pass(&c, 1);
        merged += a;
        while (P->recursive && a > 0) {
            a = rf_merge_pass(&c, 0);
            merged += a;
        }
    }
    /* sampling candidates: not selected for pruning, depth < max_depth */
    rf_key *keys = (rf_key *)malloc(sizeof(rf_key) * (L ? L : 1));
    int64_t ne = 0;
    for (int64_t l = 0; l < L; ++l) {
        double s = (double)signal[l];
        if (!rf_selected(&c, s) && c.leaf_depth[l] < P->max_depth) {
            keys[ne].s = s;
            keys[ne].idx = l;
            ++ne;
        }
    }
    int64_t k = (int64_t)floor(P->sample_frac * (double)L);
    if (k > ne) k = ne;
    qsort(keys, (size_t)ne, sizeof(rf_key), rf_cmp);
    for (int64_t j = 0; j < k; ++j) c.split[keys[j].idx] = 1;
    free(keys);
    /* capacities: at most I + k internal, L + 7k leaves */
    out->child = (int32_t *)malloc(sizeof(int32_t) * 8 * (I + k + 1));
    out->sigma = (double *)malloc(sizeof(double) * (L + 7 * k + 1));
    out->sh = (float *)malloc(sizeof(float) * 3 * c.K * (L + 7 * k + 1));
    out->depth = (int32_t *)malloc(sizeof(int32_t) * (L + 7 * k + 1));
    out->morton = (uint64_t *)malloc(sizeof(uint64_t) * (L + 7 * k + 1));
    int32_t root = I > 0 ? 0 : -1;
    rf_build(&c, root, 0, 0);
    out->merged = merged;
    out->subdivided = k;
    out->k = k;
    free(c.node_depth);
    free(c.merge);
    free(c.node_sig);
    free(c.leaf_depth);
    free(c.split);
    return 0;
}
