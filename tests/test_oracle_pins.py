"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each check is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a mis-ordered traversal) fails at
least one of them.  None of them calls the HIP library.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2307_15333_amd import synth
from tests import _ref

SQ = math.sqrt
PI = math.pi


def _root_leaf_tree(sigma, sh_dc, degree=0):
    K = (degree + 1) ** 2
    sh = np.zeros((1, 3, K), np.float64)
    sh[0, :, 0] = sh_dc
    return O.OracleTree(np.zeros((0, 8), np.int32), np.array([sigma], np.float64), sh, degree)


def _sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


# ---------------------------------------------------------------------------
# Real spherical harmonics
# ---------------------------------------------------------------------------

def _sh_cartesian(x, y, z):
    """Closed Cartesian forms of the orthonormal real SH (Condon-Shortley phase),
    derived by hand from Y = sqrt(2) K_l^m P_l^m(cos th) {cos, sin}(m phi)."""
    c1 = SQ(3 / (4 * PI))
    return np.array([
        1 / (2 * SQ(PI)),
        -c1 * y, c1 * z, -c1 * x,
        SQ(15 / (4 * PI)) * x * y,
        -SQ(15 / (4 * PI)) * y * z,
        SQ(5 / (16 * PI)) * (3 * z * z - 1),
        -SQ(15 / (4 * PI)) * x * z,
        SQ(15 / (16 * PI)) * (x * x - y * y),
        -SQ(35 / (32 * PI)) * (3 * x * x - y * y) * y,
        SQ(105 / (4 * PI)) * x * y * z,
        -SQ(21 / (32 * PI)) * y * (5 * z * z - 1),
        SQ(7 / (16 * PI)) * (5 * z ** 3 - 3 * z),
        -SQ(21 / (32 * PI)) * x * (5 * z * z - 1),
        SQ(105 / (16 * PI)) * z * (x * x - y * y),
        -SQ(35 / (32 * PI)) * (x * x - 3 * y * y) * x,
    ])


def test_sh_matches_cartesian_closed_forms():
    rng = np.random.default_rng(0)
    for _ in range(50):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        got = O.sh_basis(3, v)
        np.testing.assert_allclose(got, _sh_cartesian(*v), rtol=0, atol=1e-13)
    # poles (phi undefined) and axis directions
    for v in ([0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1, 0]):
        np.testing.assert_allclose(O.sh_basis(3, np.array(v, float)), _sh_cartesian(*v), atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for products of degree <= 6
    xs, ws = np.polynomial.legendre.leggauss(8)
    nphi = 16
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        s = math.sqrt(1 - x * x)
        for j in range(nphi):
            phi = 2 * PI * j / nphi
            Y = O.sh_basis(3, np.array([s * math.cos(phi), s * math.sin(phi), x]))
            G += np.outer(Y, Y) * w * (2 * PI / nphi)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree_prefix_and_dc():
    v = np.array([0.3, -0.4, 0.866])
    b3 = O.sh_basis(3, v)
    for deg in range(3):
        np.testing.assert_array_equal(O.sh_basis(deg, v), b3[:(deg + 1) ** 2])
    assert b3[0] == pytest.approx(0.28209479177387814, abs=1e-16)


# ---------------------------------------------------------------------------
# Compositing: closed forms (Eq. 1-2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [0.0, 0.37, 3.0, 50.0])
def test_uniform_cube_closed_form(sigma):
    """One leaf filling the root: C = (1 - e^{-sigma L}) c + e^{-sigma L} bg."""
    k0 = 0.8
    T = _root_leaf_tree(sigma, k0)
    o, d = synth.random_explicit_rays(200, seed=5, radius=3.0, spread=0.9)
    o, d = o.astype(np.float64), d.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    bg = np.array([0.2, 0.5, 0.9])
    r = O.render(T, o, d, bg=bg, t_stop=0.0)
    c = _sigmoid(k0 * 0.5 / SQ(PI))
    for i in range(o.shape[0]):
        ch = _ref.slab_chord(o[i], d[i])
        Lc = 0.0 if ch is None else ch[1] - ch[0]
        Tn = math.exp(-sigma * Lc)
        np.testing.assert_allclose(r["rgb"][i], (1 - Tn) * c + Tn * bg, atol=1e-13)


def test_uniform_subdivided_cube_equals_single_leaf():
    """A depth-2 tree with identical leaves renders like the single leaf."""
    sigma, k0 = 2.5, -0.3
    U = synth.uniform_scene(2, 1, sigma, sh_dc=k0)
    TU = O.OracleTree.from_scene(U)
    T1 = _root_leaf_tree(sigma, k0, degree=1)
    o, d = synth.random_explicit_rays(300, seed=6)
    r1 = O.render(T1, o, d, t_stop=0.0)
    r2 = O.render(TU, o, d, t_stop=0.0)
    np.testing.assert_allclose(r2["rgb"], r1["rgb"], atol=1e-12)


def test_miss_returns_background_exactly():
    s = synth.random_tree_scene(3, 1, seed=1)
    T = O.OracleTree.from_scene(s)
    o = np.array([[3.0, 3.0, 3.0], [0.0, 0.0, 5.0]])
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])   # pointing away
    bg = (0.1, 0.7, 0.3)
    r = O.render(T, o, d, bg=bg)
    np.testing.assert_array_equal(r["rgb"], np.array([bg, bg]))
    assert (r["nseg"] == 0).all()


def test_colour_equal_background_is_invariant():
    """All leaf colours = bg => C = bg for any densities (weights + T_end = 1)."""
    s = synth.random_tree_scene(4, 2, seed=2, sigma_max=30.0)
    sh = np.zeros_like(s.sh64)           # sigmoid(0) = 0.5
    T = O.OracleTree.from_scene(s, sh=sh)
    o, d = synth.random_explicit_rays(500, seed=7)
    r = O.render(T, o, d, bg=0.5, t_stop=0.0)
    np.testing.assert_allclose(r["rgb"], 0.5, atol=1e-14)


def test_weights_sum_with_transmittance_is_one():
    """Identity colour 1 and bg 0: C = 1 - exp(-sum sigma delta); also sum of
    the per-leaf SUM-signal over one ray equals C."""
    s = synth.random_tree_scene(4, 0, seed=3, sigma_max=6.0)
    sh = np.full((s.n_leaves, 3, 1), 1.0 / 0.28209479177387814)   # c = 1 exactly-ish
    T = O.OracleTree.from_scene(s, sh=sh)
    o, d = synth.random_explicit_rays(40, seed=8)
    for i in range(o.shape[0]):
        oi, di = o[i:i + 1].astype(np.float64), d[i:i + 1].astype(np.float64)
        r = O.render(T, oi, di, bg=0.0, t_stop=0.0, activation="identity", signal=True,
                     signal_mode="sum")
        leaf, delta = O.ray_segments(T, oi[0], di[0])
        tau = (np.maximum(s.sigma64[leaf], 0) * delta).sum()
        np.testing.assert_allclose(r["rgb"][0], 1 - math.exp(-tau), atol=1e-12)
        np.testing.assert_allclose(r["sig"].sum(), 1 - math.exp(-tau), atol=1e-12)


def test_two_leaf_weights_closed_form():
    """Depth-1 uniform tree, ray along +x through y,z > 0 half: weights of the
    two leaves are 1-e^{-s1 d1} and e^{-s1 d1}(1-e^{-s2 d2})."""
    U = synth.uniform_scene(1, 0, 1.0)
    sig = np.zeros(8)
    # octant with x low, y high, z high is 6; x high: 7
    sig[6], sig[7] = 0.7, 2.0
    T = O.OracleTree(U.child, sig, U.sh64, 0)
    o = np.array([[-3.0, 0.4, 0.6]])
    d = np.array([[1.0, 0.0, 0.0]])
    r = O.render(T, o, d, t_stop=0.0, signal=True)
    w1 = 1 - math.exp(-0.7)
    w2 = math.exp(-0.7) * (1 - math.exp(-2.0))
    assert r["sig"][6] == pytest.approx(w1, abs=1e-15)
    assert r["sig"][7] == pytest.approx(w2, abs=1e-15)
    assert r["sig"][[0, 1, 2, 3, 4, 5]].max() == 0.0


# ---------------------------------------------------------------------------
# Traversal: textbook special case and brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("depth", [1, 3, 4])
def test_traversal_matches_dense_grid_dda(depth):
    U = synth.uniform_scene(depth, 0, 1.0)
    T = O.OracleTree.from_scene(U)
    n = 1 << depth
    cell_to_leaf = {tuple(c): i for i, c in enumerate(U.leaf_ijk)}
    o, d = synth.random_explicit_rays(150, seed=9 + depth)
    o, d = o.astype(np.float64), d.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for i in range(o.shape[0]):
        leaf, delta = O.ray_segments(T, o[i], d[i])
        cells, lens = _ref.dda_grid(o[i], d[i], n)
        exp_leaf = [cell_to_leaf[c] for c, ln in zip(cells, lens) if ln > 1e-12]
        exp_len = [ln for ln in lens if ln > 1e-12]
        keep = delta > 1e-12
        assert list(leaf[keep]) == exp_leaf
        np.testing.assert_allclose(delta[keep], exp_len, atol=1e-12)


def test_ray_in_a_cell_plane_belongs_to_the_upper_cell():
    """Leaves tile the root: a ray lying in the plane between two cells crosses
    one of them (half-open cells, the upper one), never both; a ray on the
    root's upper face belongs to the last cell."""
    U = synth.uniform_scene(1, 0, 1.0)
    sig = np.arange(1.0, 9.0)           # distinct densities per octant
    T = O.OracleTree(U.child, sig, U.sh64, 0)
    d = np.array([1.0, 0.0, 0.0])
    cases = [((-3.0, 0.0, 0.0), [6, 7]),      # y = z = 0: upper y, upper z octants (6, 7)
             ((-3.0, -0.5, 0.0), [4, 5]),     # z = 0 only
             ((-3.0, 1.0, -1.0), [2, 3]),     # y on the root's upper face, z on the lower face
             ((-3.0, 1.0, 1.0), [6, 7])]      # the upper root edge
    for o, want in cases:
        leaf, delta = O.ray_segments(T, np.array(o), d)
        assert list(leaf) == want, (o, leaf)
        np.testing.assert_allclose(delta, [1.0, 1.0], atol=1e-15)
    # a diagonal ray through cell corners: only positive-length segments, total = chord
    o = np.array([-3.0, -3.0, -3.0])
    dd = np.ones(3) / np.sqrt(3.0)
    leaf, delta = O.ray_segments(O.OracleTree.from_scene(synth.uniform_scene(3, 0, 1.0)), o, dd)
    assert len(leaf) == 8 and abs(delta.sum() - 2 * np.sqrt(3.0)) < 1e-12


def test_segments_sum_to_chord_and_match_ray_marching():
    s = synth.random_tree_scene(5, 0, seed=4)
    T = O.OracleTree.from_scene(s)
    o, d = synth.random_explicit_rays(25, seed=12)
    o, d = o.astype(np.float64), d.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    h = 2e-4
    for i in range(o.shape[0]):
        leaf, delta = O.ray_segments(T, o[i], d[i])
        ch = _ref.slab_chord(o[i], d[i])
        assert delta.sum() == pytest.approx(ch[1] - ch[0], abs=1e-12)
        # midpoint marching: per-leaf path length within a few steps
        ts = np.arange(ch[0] + h / 2, ch[1], h)
        hits = {}
        for t in ts:
            l = _ref.locate_leaf(s.child, o[i] + t * d[i])
            hits[l] = hits.get(l, 0.0) + h
        seg = {}
        for l, dl in zip(leaf, delta):
            seg[int(l)] = seg.get(int(l), 0.0) + dl
        for l in set(hits) | set(seg):
            assert abs(hits.get(l, 0.0) - seg.get(l, 0.0)) <= 2.5 * h
        # front-to-back order: the first marched leaf is the first segment
        assert _ref.locate_leaf(s.child, o[i] + ts[0] * d[i]) == leaf[0]
        # optical depth converges
        tau_seg = (s.sigma64[leaf] * delta).sum()
        tau_march = sum(s.sigma64[l] * v for l, v in hits.items())
        assert abs(tau_seg - tau_march) < 4 * h * s.sigma64.max()


def test_subdividing_a_leaf_into_copies_leaves_pixels_unchanged():
    s = synth.random_tree_scene(4, 2, seed=5, sigma_max=12.0)
    T = O.OracleTree.from_scene(s)
    rng = np.random.default_rng(0)
    cams = synth.cameras([(20.0, 35.0, 3.5, 24, 24)])
    o, d = O.camera_rays(cams)
    base = O.render(T, o, d, t_stop=0.0)["rgb"]
    for leaf in rng.choice(s.n_leaves, 6, replace=False):
        ld = list(s.leaf_depth.astype(np.int64))
        lijk = [tuple(x) for x in s.leaf_ijk]
        sig = list(s.sigma64)
        sh = list(s.sh64)
        d0, c0 = ld.pop(leaf), lijk.pop(leaf)
        v_sig, v_sh = sig.pop(leaf), sh.pop(leaf)
        for oc in range(8):
            ld.append(d0 + 1)
            lijk.append(tuple(np.array(c0) * 2 + synth.OCT[oc]))
            sig.append(v_sig)
            sh.append(v_sh)
        ld, lijk = np.array(ld), np.array(lijk)
        child, order = synth.tree_from_cells(ld, lijk, int(ld.max()))
        T2 = O.OracleTree(child, np.array(sig)[order], np.array(sh)[order], s.degree)
        r = O.render(T2, o, d, t_stop=0.0)["rgb"]
        np.testing.assert_allclose(r, base, atol=1e-12)


# ---------------------------------------------------------------------------
# Early termination and the straddle branches
# ---------------------------------------------------------------------------

def test_early_stop_branches():
    """Single leaf along x with sigma*L just above / below -ln(t_stop)."""
    thr = -math.log(1e-4)
    U = synth.uniform_scene(1, 0, 1.0)
    o = np.array([[-3.0, 0.5, 0.5]])
    d = np.array([[1.0, 0.0, 0.0]])
    for tau_total in (thr + 5e-4, thr + 0.5, thr - 0.5):
        sig = np.full(8, tau_total / 2.0)     # the ray crosses two leaves of length 1
        T = O.OracleTree(U.child, sig, np.zeros((8, 3, 1)), 0)
        r = O.render(T, o, d, bg=1.0, t_stop=1e-4, margin=1e-3)
        # the ray ends after its second segment whichever rule applies, so the
        # branches coincide and no straddle is reported
        assert not r["straddle"][0]
        assert r["nseg"][0] == 2
        # the stop happens after the second segment in every branch (no third segment),
        # so all three colours agree with the full composite
        full = O.render(T, o, d, bg=1.0, t_stop=0.0)["rgb"]
        np.testing.assert_allclose(r["rgb"], full, atol=1e-15)
    # a three-leaf ray where the early branch stops before the last segment
    U2 = synth.uniform_scene(2, 0, 1.0)
    o = np.array([[-3.0, 0.3, 0.3]])
    sig = np.zeros(U2.n_leaves)
    path, lens = O.ray_segments(O.OracleTree.from_scene(U2), o[0], d[0])
    assert len(path) == 4
    sig[path[0]] = (thr - 4e-4) / 0.5
    sig[path[1]] = 1e-4 / 0.5        # small step: crosses only the early threshold
    sig[path[2]] = 3.0
    sh = np.zeros((U2.n_leaves, 3, 1))
    sh[path[2], :, 0] = 3.0
    T = O.OracleTree(U2.child, sig, sh, 0)
    r = O.render(T, o, d, bg=0.0, t_stop=1e-4, margin=1e-3)
    assert r["straddle"][0]
    assert r["nseg"][0] == 3
    assert not np.allclose(r["rgb_early"], r["rgb_late"], atol=1e-9)
    np.testing.assert_allclose(r["rgb"], r["rgb_late"], atol=1e-15)


# ---------------------------------------------------------------------------
# Gradient: central finite differences in FP64
# ---------------------------------------------------------------------------

def test_backward_matches_central_differences():
    s = synth.random_tree_scene(3, 2, seed=7, sigma_max=5.0)
    sig = s.sigma64 + 0.05        # keep away from the ReLU kink
    sh = s.sh64.copy()
    cams = synth.cameras([(35.0, 25.0, 3.0, 16, 16)])
    o, d = O.camera_rays(cams)
    rng = np.random.default_rng(1)
    g = rng.normal(size=(o.shape[0], 3))
    bg = np.array([0.3, 0.6, 0.9])
    T = O.OracleTree(s.child, sig, sh, s.degree)
    gs, gh = O.backward(T, o, d, g, bg=bg, t_stop=0.0)

    def loss(sig_, sh_):
        r = O.render(O.OracleTree(s.child, sig_, sh_, s.degree), o, d, bg=bg, t_stop=0.0)
        return float((r["rgb"] * g).sum())

    # central differences carry O(h^2) truncation and ~eps*|loss|/h rounding
    # error (|loss| ~ 30 here): h = 1e-5 keeps both below ~1e-9
    h = 1e-5
    hit = np.where(np.abs(gs) > 1e-3)[0]
    assert hit.shape[0] > 20
    for l in rng.choice(hit, 12, replace=False):
        a, b = sig.copy(), sig.copy()
        a[l] += h
        b[l] -= h
        fd = (loss(a, sh) - loss(b, sh)) / (2 * h)
        assert fd == pytest.approx(gs[l], rel=1e-6, abs=1e-8)
    flat = np.abs(gh).reshape(-1)
    idx = rng.choice(np.where(flat > 1e-4)[0], 12, replace=False)
    for j in idx:
        a, b = sh.copy().reshape(-1), sh.copy().reshape(-1)
        a[j] += h
        b[j] -= h
        fd = (loss(sig, a.reshape(sh.shape)) - loss(sig, b.reshape(sh.shape))) / (2 * h)
        assert fd == pytest.approx(gh.reshape(-1)[j], rel=1e-6, abs=1e-8)


def test_backward_with_early_stop_matches_central_differences():
    """With early termination (t_stop = 1e-4) the render is the sum truncated
    after the segment that takes S past ln 1e4 (plus the background term), and
    the adjoint must stop at that same segment.  On rays whose stop decision is
    far from the threshold (no straddle within 1e-2 of optical depth, far more
    than a perturbation of h moves S), central differences of the truncated
    render pin the gradient of every leaf's density and of sampled SH
    coefficients; leaves past or at the stop of some rays are included, so
    adjoining one segment too many or too few fails."""
    s = synth.random_tree_scene(3, 2, seed=17, sigma_max=12.0)
    sig = s.sigma64 + 0.05
    sh = s.sh64.copy()
    cams = synth.cameras([(35.0, 25.0, 3.0, 16, 16), (-120.0, -30.0, 3.2, 16, 16)])
    o, d = O.camera_rays(cams)
    bg = np.array([0.3, 0.6, 0.9])
    T = O.OracleTree(s.child, sig, sh, s.degree)
    r = O.render(T, o, d, bg=bg, t_stop=1e-4, margin=1e-2)
    full = O.render(T, o, d, bg=bg, t_stop=0.0)
    keep = ~r["straddle"].astype(bool)
    o, d = o[keep], d[keep]
    stopped = (r["nseg"] < full["nseg"])[keep]
    assert stopped.sum() > 50 and (~stopped).sum() > 20
    rng = np.random.default_rng(3)
    g = rng.normal(size=(o.shape[0], 3))
    gs, gh = O.backward(T, o, d, g, bg=bg, t_stop=1e-4)
    gs0, gh0 = O.backward(T, o, d, g, bg=bg, t_stop=0.0)
    # the truncation changes the gradient of many leaves, each by far more than
    # the differences' error (the terms past the stop carry T < 1e-4)
    moved = np.where(np.abs(gs - gs0) > 1e-6)[0]
    assert moved.shape[0] > 10

    def loss(sig_, sh_):
        rr = O.render(O.OracleTree(s.child, sig_, sh_, s.degree), o, d, bg=bg, t_stop=1e-4, margin=0.0)
        return float((rr["rgb"] * g).sum())

    h = 1e-5
    for l in range(sig.shape[0]):
        a, b = sig.copy(), sig.copy()
        a[l] += h
        b[l] -= h
        fd = (loss(a, sh) - loss(b, sh)) / (2 * h)
        assert fd == pytest.approx(gs[l], rel=1e-6, abs=1e-8), l
    # SH: coefficients of the leaves whose gradient the truncation moved, and others
    flat = np.abs(gh).reshape(-1)
    K3 = 3 * (s.degree + 1) ** 2
    on_moved = np.concatenate([np.arange(l * K3, (l + 1) * K3) for l in moved])
    cand = np.union1d(rng.choice(on_moved, 16, replace=False), rng.choice(np.where(flat > 1e-4)[0], 16, replace=False))
    for j in cand:
        a, b = sh.copy().reshape(-1), sh.copy().reshape(-1)
        a[j] += h
        b[j] -= h
        fd = (loss(sig, a.reshape(sh.shape)) - loss(sig, b.reshape(sh.shape))) / (2 * h)
        assert fd == pytest.approx(gh.reshape(-1)[j], rel=1e-6, abs=1e-8), j


def test_backward_single_leaf_closed_form():
    """One leaf: dC/dk = w c (1-c) Y(d); dC/dsigma = L e^{-sigma L}(c - bg)."""
    sigma, k0 = 1.3, 0.4
    T = _root_leaf_tree(sigma, k0)
    o = np.array([[-3.0, 0.1, -0.2]])
    d = np.array([[1.0, 0.0, 0.0]])
    bg = np.array([0.9, 0.2, 0.4])
    g = np.array([[1.0, -0.5, 0.25]])
    gs, gh = O.backward(T, o, d, g, bg=bg, t_stop=0.0)
    Lc = 2.0
    c = _sigmoid(k0 * 0.5 / SQ(PI))
    w = 1 - math.exp(-sigma * Lc)
    exp_sig = sum(g[0, ch] * Lc * math.exp(-sigma * Lc) * (c - bg[ch]) for ch in range(3))
    assert gs[0] == pytest.approx(exp_sig, rel=1e-13)
    for ch in range(3):
        assert gh[0, ch, 0] == pytest.approx(g[0, ch] * w * c * (1 - c) * 0.5 / SQ(PI), rel=1e-13)


def test_zero_residual_gives_zero_gradient_and_relu_kink():
    s = synth.random_tree_scene(3, 1, seed=8)
    sig = s.sigma64.copy()
    sig[::3] = -1.0                      # negative raw density: no gradient
    T = O.OracleTree(s.child, sig, s.sh64, s.degree)
    o, d = synth.random_explicit_rays(64, seed=13)
    gs, gh = O.backward(T, o, d, np.zeros((64, 3)), t_stop=0.0)
    assert not gs.any() and not gh.any()
    gs, gh = O.backward(T, o, d, np.ones((64, 3)), t_stop=0.0)
    assert not gs[::3].any()


# ---------------------------------------------------------------------------
# Storage rounding (IEEE-754 round to nearest even)
# ---------------------------------------------------------------------------

def test_round_storage_matches_library_casts():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-8, 5, 2000),
                        [0.0, -0.0, 65504.0, 65520.0, 1e-8, 6.1e-5, 2.0 ** -24, 2.0 ** -25,
                         1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11]])
    np.testing.assert_array_equal(O.round_storage(x, "f16"), x.astype(np.float16).astype(np.float64))
    np.testing.assert_array_equal(O.round_storage(x, "f32"), x.astype(np.float32).astype(np.float64))
    # bf16: on FP32-representable inputs, RNE of the upper 16 bits of the FP32 pattern
    x32 = x.astype(np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    rounded = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    exp = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(O.round_storage(x32.astype(np.float64), "bf16"), exp)


# ---------------------------------------------------------------------------
# Refinement (Eq. 3 / Eq. 4, Alg. 1)
# ---------------------------------------------------------------------------

def _check_refined_topology(s, R, signal, tau, frac, maxd):
    child, depth, ijk, merged, k = _ref.refine_by_leaf_list(s, signal, tau, frac, maxd)
    np.testing.assert_array_equal(R["child"], child)
    np.testing.assert_array_equal(R["depth"], depth)
    np.testing.assert_array_equal(R["morton"], synth.morton3(ijk))
    assert R["merged"] == merged and R["k"] == k
    L0, L1 = s.n_leaves, R["sigma"].shape[0]
    assert L1 == L0 - 7 * merged + 7 * k
    assert ((2.0 / 2.0 ** R["depth"]) ** 3).sum() == pytest.approx(8.0, abs=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_refine_matches_leaf_list_construction(seed):
    s = synth.random_tree_scene(3, 1, seed=seed, p_split=0.5)
    rng = np.random.default_rng(seed)
    signal = rng.uniform(0, 1, s.n_leaves).astype(np.float32)
    signal[rng.random(s.n_leaves) < 0.5] *= 1e-3        # many prunable leaves
    tau, frac, maxd = 1e-3, 0.1, 4
    T = O.OracleTree.from_scene(s)
    R = O.refine(T, signal, tau=tau, sample_frac=frac, max_depth=maxd)
    _check_refined_topology(s, R, signal, tau, frac, maxd)


def test_refine_values_mean_and_copy():
    s = synth.random_tree_scene(3, 2, seed=21, p_split=0.5)
    rng = np.random.default_rng(2)
    signal = rng.uniform(0.5, 1, s.n_leaves).astype(np.float32)
    # make exactly one 8-leaf group prunable
    groups = {}
    for i in range(s.n_leaves):
        groups.setdefault((s.leaf_depth[i] - 1, tuple(s.leaf_ijk[i] >> 1)), []).append(i)
    full = [m for m in groups.values() if len(m) == 8]
    grp = full[0]
    signal[grp] = 0.0
    for storage in ("f32", "f16", "bf16"):
        T = O.OracleTree.from_scene(s)
        R = O.refine(T, signal, tau=0.0, sample_frac=0.05, max_depth=5, storage=storage)
        assert R["merged"] == 1
        # the merged leaf: depth of the parent, value = FP64 mean rounded once
        pd = s.leaf_depth[grp[0]] - 1
        pm = synth.morton3(s.leaf_ijk[grp[0]] >> 1)
        j = np.where((R["depth"] == pd) & (R["morton"] == pm))[0]
        assert j.shape[0] == 1
        j = j[0]
        assert R["sigma"][j] == O.round_storage(np.array([s.sigma64[grp].mean()]), storage)[0]
        np.testing.assert_array_equal(
            R["sh"][j].astype(np.float64),
            O.round_storage(s.sh64[grp].mean(axis=0), storage))
        # split leaves: 8 bit-exact copies (after storage rounding of the parent)
        k = R["k"]
        order = sorted(np.where(signal > 0.0)[0].tolist(), key=lambda i: (-signal[i], i))[:k]
        for i in order:
            kids = np.where((R["depth"] == s.leaf_depth[i] + 1) &
                            ((R["morton"] >> np.uint64(3)) == synth.morton3(s.leaf_ijk[i])))[0]
            assert kids.shape[0] == 8
            for kk in kids:
                assert R["sigma"][kk] == O.round_storage(np.array([s.sigma64[i]]), storage)[0]


def test_refine_merge_of_equal_children_inverts_subdivision():
    """Merging 8 equal children restores the parent; the render is unchanged."""
    s = synth.random_tree_scene(3, 1, seed=30, p_split=0.4)
    T = O.OracleTree.from_scene(s)
    sig1 = np.ones(s.n_leaves, np.float32)
    leaf = int(np.argmax(s.leaf_depth < 3))
    sig1[leaf] = 2.0
    R1 = O.refine(T, sig1, tau=0.0, sample_frac=1.0 / s.n_leaves + 1e-9, max_depth=4)
    assert R1["k"] == 1 and R1["merged"] == 0
    T1 = O.OracleTree(R1["child"], R1["sigma"], R1["sh"], s.degree)
    sig2 = np.ones(R1["sigma"].shape[0], np.float32)
    kids = np.where(R1["depth"] == s.leaf_depth[leaf] + 1)[0]
    new = [kk for kk in kids if (R1["morton"][kk] >> np.uint64(3)) == synth.morton3(s.leaf_ijk[leaf])]
    sig2[new] = 0.0
    R2 = O.refine(T1, sig2, tau=0.0, sample_frac=0.0, max_depth=4)
    assert R2["merged"] == 1
    np.testing.assert_array_equal(R2["child"], s.child)
    np.testing.assert_array_equal(R2["sigma"], s.sigma64.astype(np.float32).astype(np.float64))
    o, d = synth.random_explicit_rays(100, seed=3)
    a = O.render(T, o, d, t_stop=0.0)["rgb"]
    b = O.render(O.OracleTree(R2["child"], R2["sigma"], R2["sh"], s.degree), o, d, t_stop=0.0)["rgb"]
    np.testing.assert_allclose(a, b, atol=1e-6)


def test_refine_ties_threshold_and_topk():
    s = synth.uniform_scene(2, 0, 1.0)
    T = O.OracleTree.from_scene(s)
    # prune comparison at an exactly representable tie: s <= tau selects it
    signal = np.full(64, 0.25, np.float32)
    R = O.refine(T, signal, tau=0.25, sample_frac=0.0, max_depth=3, prune_le=True)
    assert R["merged"] == 8
    R = O.refine(T, signal, tau=0.25, sample_frac=0.0, max_depth=3, prune_le=False)
    assert R["merged"] == 0
    # top-k with equal keys: the lower DFS index wins
    signal = np.full(64, 0.5, np.float32)
    R = O.refine(T, signal, tau=0.1, sample_frac=3 / 64, max_depth=3)
    assert R["k"] == 3
    assert (R["depth"][:24] == 3).all() and (R["depth"][24:] == 2).all()
    # max_depth excludes candidates
    R = O.refine(T, signal, tau=0.1, sample_frac=0.5, max_depth=2)
    assert R["k"] == 0 and R["sigma"].shape[0] == 64


def test_refine_recursive_climbs_hierarchy():
    s = synth.uniform_scene(3, 0, 1.0)
    T = O.OracleTree.from_scene(s)
    signal = np.zeros(512, np.float32)
    R = O.refine(T, signal, tau=0.0, sample_frac=0.0, max_depth=4, recursive=False)
    assert R["merged"] == 64 and R["sigma"].shape[0] == 64
    R = O.refine(T, signal, tau=0.0, sample_frac=0.0, max_depth=4, recursive=True)
    assert R["merged"] == 64 + 8 + 1
    assert R["sigma"].shape[0] == 1 and R["child"].shape[0] == 0


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_refine_recursive_merge_values_are_means_of_level_means(storage):
    """Recursive pruning applies Eq. 3 level by level: a node whose children
    were merged in the same pass gets the mean of their (already rounded)
    means, not the mean of all the leaves below it.  Tree: the root's octant 0
    is an internal node with 8 leaves, octants 1-7 are leaves; every value is
    distinct.  Non-recursive: only the inner group merges; recursive: the
    whole tree collapses to one leaf."""
    rng = np.random.default_rng(40)
    child = np.array([[1] + [-1 - (8 + j) for j in range(7)], [-1 - j for j in range(8)]], np.int32)
    vals = rng.uniform(-3.0, 3.0, size=(15, 1 + 3 * 4))
    vals = O.round_storage(vals, storage)             # stored values
    T = O.OracleTree(child, vals[:, 0].copy(), vals[:, 1:].reshape(15, 3, 4).copy(), 1)
    sig = np.zeros(15, np.float32)

    def mean8(rows):
        return O.round_storage(np.array([math.fsum(rows[:, j]) / 8.0 for j in range(rows.shape[1])]), storage)

    inner = mean8(vals[:8])
    R = O.refine(T, sig, tau=0.0, sample_frac=0.0, max_depth=4, recursive=False, storage=storage)
    assert R["merged"] == 1 and R["sigma"].shape[0] == 8
    np.testing.assert_array_equal(np.concatenate([R["sigma"][:1], R["sh"][0].reshape(-1)]), inner)
    np.testing.assert_array_equal(R["sigma"][1:], vals[8:, 0])
    R = O.refine(T, sig, tau=0.0, sample_frac=0.0, max_depth=4, recursive=True, storage=storage)
    assert R["merged"] == 2 and R["sigma"].shape[0] == 1 and R["child"].shape[0] == 0
    want = mean8(np.vstack([inner[None, :], vals[8:]]))
    np.testing.assert_array_equal(np.concatenate([R["sigma"], R["sh"][0].reshape(-1)]), want)
    # the mean over all 15 leaves (or over the 8 top-level cells without the
    # inner rounding) is a different value: the pin tells the readings apart
    flat = O.round_storage(vals.mean(axis=0), storage)
    assert np.abs(flat - want).max() > 0.05


def test_refine_reinit_zeroes_only_new_leaves():
    """The fusion-disabled ablation: the same topology; merged leaves and the
    children of split leaves start at zero, untouched leaves keep their values."""
    s = synth.random_tree_scene(3, 1, seed=31, p_split=0.5)
    rng = np.random.default_rng(5)
    signal = rng.uniform(0.5, 1.0, s.n_leaves).astype(np.float32)
    groups = {}
    for i in range(s.n_leaves):
        groups.setdefault((s.leaf_depth[i] - 1, tuple(s.leaf_ijk[i] >> 1)), []).append(i)
    grp = [m for m in groups.values() if len(m) == 8][0]
    signal[grp] = 0.0
    T = O.OracleTree.from_scene(s)
    A = O.refine(T, signal, tau=0.0, sample_frac=0.05, max_depth=5)
    B = O.refine(T, signal, tau=0.0, sample_frac=0.05, max_depth=5, reinit=True)
    np.testing.assert_array_equal(A["child"], B["child"])
    np.testing.assert_array_equal(A["depth"], B["depth"])
    fresh = np.zeros(A["sigma"].shape[0], bool)
    old_key = {(int(d), int(m)) for d, m in zip(s.leaf_depth, synth.morton3(s.leaf_ijk))}
    for j, (d, m) in enumerate(zip(A["depth"], A["morton"])):
        fresh[j] = (int(d), int(m)) not in old_key
    assert fresh.sum() == 1 + 8 * A["k"]
    assert not B["sigma"][fresh].any() and not B["sh"][fresh].any()
    np.testing.assert_array_equal(B["sigma"][~fresh], A["sigma"][~fresh])
    np.testing.assert_array_equal(B["sh"][~fresh], A["sh"][~fresh])


def test_refine_root_leaf():
    T = _root_leaf_tree(1.0, 0.5, degree=1)
    R = O.refine(T, np.array([0.9], np.float32), tau=0.1, sample_frac=1.0, max_depth=2)
    assert R["k"] == 1 and R["child"].shape == (1, 8)
    np.testing.assert_array_equal(R["child"][0], -1 - np.arange(8))


# ---------------------------------------------------------------------------
# Cameras
# ---------------------------------------------------------------------------

def test_camera_rays_principal_and_fov():
    cam = synth.cameras([(30.0, 20.0, 4.0, 1, 1)])
    o, d = O.camera_rays(cam)
    np.testing.assert_allclose(d[0], -o[0] / np.linalg.norm(o[0]), atol=1e-7)
    assert np.linalg.norm(o[0]) == pytest.approx(4.0, rel=1e-7)
    # horizontal FOV: the two edge pixel rays of a wide row span 40 degrees (up to
    # half a pixel at each end)
    W = 2001
    cam = synth.cameras([(10.0, -15.0, 4.0, W, 1)])
    o, d = O.camera_rays(cam, np.zeros(2, np.int32), np.array([0, W - 1], np.int32))
    ang = math.degrees(math.acos(np.clip(d[0] @ d[1], -1, 1)))
    half_px = math.degrees(2 * math.atan(math.tan(math.radians(20)) * (W - 1) / W))
    assert ang == pytest.approx(half_px, abs=1e-5)
