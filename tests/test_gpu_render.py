"""Forward renderer and fused signal on the GPU versus the FP64 oracle.

Tolerances (per channel, absolute): 1e-5 for FP32 leaves; 2e-3 for FP16/BF16
leaves measured against the FP64 generator values.  A ray whose stop decision
sits within the oracle's straddle window may match either stopping branch.
The per-leaf MAX signal must lie within [sig_lo - 1e-5, sig_hi + 1e-5], the
signals of the early and late stopping rules.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2307_15333_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 2e-3


def _core():
    from paper_2307_15333_amd import core
    return core


def rgb_err(gpu, ref):
    g = np.asarray(gpu, np.float64)
    e = np.minimum(np.abs(g - ref["rgb"]).max(1),
                   np.minimum(np.abs(g - ref["rgb_early"]).max(1), np.abs(g - ref["rgb_late"]).max(1)))
    return e


def oracle_tree(scene, storage="f32"):
    if storage == "f32":
        return O.OracleTree.from_scene(scene, sigma=scene.sigma.astype(np.float64))
    sig = O.round_storage(scene.sigma.astype(np.float64), storage)
    sh = O.round_storage(scene.sh32.astype(np.float64), storage)
    return O.OracleTree(scene.child, sig, sh, scene.degree)


@pytest.fixture(scope="module")
def sphere():
    return synth.sphere_scene()


def _render(scene, rays, storage="f32", **kw):
    core = _core()
    tree = core.Octree.from_scene(scene, storage)
    L = tree.n_leaves
    sig = torch.zeros(L, dtype=torch.float32, device="cuda")
    rgb, ns = tree.render(rays, nseg=True, signal=sig, **kw)
    torch.cuda.synchronize()
    out = rgb.cpu().numpy(), ns.cpu().numpy(), sig.cpu().numpy()
    tree.close()
    return out


@pytest.mark.parametrize("t_stop", [1e-4, 0.0])
def test_sphere_fp32_parity(sphere, t_stop):
    core = _core()
    cams = synth.sphere_camera()
    rgb, ns, sig = _render(sphere, core.Rays.cameras(cams), t_stop=t_stop)
    o, d = O.camera_rays(cams)
    ref = O.render(oracle_tree(sphere), o, d, t_stop=t_stop, signal=True)
    e = rgb_err(rgb, ref)
    print(f"sphere t_stop={t_stop}: max err {e.max():.3e} mean {e.mean():.3e} straddle {ref['straddle'].sum()}")
    assert e.max() <= TOL32
    assert np.all(sig >= ref["sig_lo"] - TOL32) and np.all(sig <= ref["sig_hi"] + TOL32)
    same = (ns == ref["nseg"]) | ref["straddle"]
    assert same.mean() >= 0.999, same.mean()


def test_signal_sum_mode(sphere):
    core = _core()
    cams = synth.sphere_camera()
    tree = core.Octree.from_scene(sphere)
    sig = torch.zeros(tree.n_leaves, dtype=torch.float32, device="cuda")
    tree.accumulate_signal(core.Rays.cameras(cams), sig, t_stop=0.0, signal_mode="sum")
    o, d = O.camera_rays(cams)
    ref = O.render(oracle_tree(sphere), o, d, t_stop=0.0, signal=True, signal_mode="sum")
    got = sig.cpu().numpy()
    np.testing.assert_allclose(got, ref["sig"], atol=1e-4, rtol=1e-5)
    tree.close()


@pytest.mark.parametrize("w,h", [(61, 37), (1, 1), (8, 8), (9, 17), (130, 3)])
def test_ragged_images(sphere, w, h):
    core = _core()
    cams = synth.cameras([(30.0, 20.0, 4.0, w, h), (200.0, -40.0, 3.5, w, h)])
    rgb, ns, sig = _render(sphere, core.Rays.cameras(cams))
    o, d = O.camera_rays(cams)
    ref = O.render(oracle_tree(sphere), o, d, signal=True)
    assert rgb_err(rgb, ref).max() <= TOL32


def test_pixel_list_mode(sphere):
    core = _core()
    views = synth.training_views(n=7)
    ci, pi = synth.pixel_batch(7, 64, 64, 3001, seed=5)
    rgb, ns, sig = _render(sphere, core.Rays.pixels(views, ci, pi))
    o, d = O.camera_rays(views, ci, pi)
    ref = O.render(oracle_tree(sphere), o, d, signal=True)
    assert rgb_err(rgb, ref).max() <= TOL32
    assert np.all(sig >= ref["sig_lo"] - TOL32) and np.all(sig <= ref["sig_hi"] + TOL32)


def _edge_rays():
    o, d = synth.random_explicit_rays(2000, seed=11, radius=2.5, spread=1.3)
    extra_o = np.array([
        [0.1, 0.2, 0.3], [0.0, 0.0, 0.0],              # inside the cube
        [-3.0, 0.0, 0.0], [-3.0, 0.5, 0.25],           # along lattice planes
        [-3.0, 1.0, 1.0], [0.0, -3.0, 0.0],            # along an edge of the root, an axis
        [5.0, 5.0, 5.0], [-3.0, 0.3, -0.7],            # misses; axis-aligned inside
        [-3.0, -3.0, -3.0],                            # through the corner diagonal
    ], np.float32)
    extra_d = np.array([
        [0.3, -0.5, 0.8], [1.0, 0.0, 0.0],
        [1.0, 0.0, 0.0], [1.0, 0.0, 0.0],
        [1.0, 0.0, 0.0], [0.0, 1.0, 0.0],
        [1.0, 0.0, 0.0], [1.0, 0.0, 0.0],
        [1.0, 1.0, 1.0],
    ], np.float32)
    extra_d /= np.linalg.norm(extra_d, axis=1, keepdims=True)
    return np.concatenate([o, extra_o]), np.concatenate([d, extra_d])


@pytest.mark.parametrize("seed", [0, 1])
def test_explicit_rays_random_trees(seed):
    core = _core()
    s = synth.random_tree_scene(6, 3, seed=seed, p_split=0.42, sigma_max=20.0)
    o, d = _edge_rays()
    rgb, ns, sig = _render(s, core.Rays.explicit(o, d), bg=(0.2, 0.4, 0.6))
    d64 = d.astype(np.float64)
    ref = O.render(oracle_tree(s), o.astype(np.float64), d64, bg=(0.2, 0.4, 0.6), signal=True)
    e = rgb_err(rgb, ref)
    print(f"random tree {s.n_leaves} leaves: max err {e.max():.3e}")
    assert e.max() <= TOL32
    assert np.all(sig >= ref["sig_lo"] - TOL32) and np.all(sig <= ref["sig_hi"] + TOL32)


def test_degenerate_trees():
    core = _core()
    o, d = _edge_rays()
    for s in (synth.uniform_scene(0, 1, 3.0, sh_dc=0.7),      # the root is a leaf
              synth.uniform_scene(4, 2, 6.0, seed=3)):         # depth-uniform
        rgb, ns, sig = _render(s, core.Rays.explicit(o, d))
        ref = O.render(oracle_tree(s), o.astype(np.float64), d.astype(np.float64), signal=True)
        assert rgb_err(rgb, ref).max() <= TOL32


def test_empty_batches(sphere):
    core = _core()
    tree = core.Octree.from_scene(sphere)
    rays = core.Rays.explicit(np.zeros((0, 3)), np.zeros((0, 3)))
    rgb = tree.render(rays)
    assert rgb.shape == (0, 3)
    cams = synth.sphere_camera()
    r = core.Rays.cameras(cams)
    r.struct.n_cams = 0
    tree.render(r)
    torch.cuda.synchronize()
    tree.close()


def test_render_is_deterministic(sphere):
    core = _core()
    cams = synth.cameras([(30.0, 20.0, 4.0, 64, 64), (100.0, 10.0, 4.0, 64, 64)])
    tree = core.Octree.from_scene(sphere)
    rays = core.Rays.cameras(cams)
    outs = []
    for _ in range(3):
        sig = torch.zeros(tree.n_leaves, dtype=torch.float32, device="cuda")
        rgb = tree.render(rays, signal=sig)
        outs.append((rgb.cpu().numpy(), sig.cpu().numpy()))
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])
    tree.close()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_reduced_precision_leaves(sphere, storage):
    core = _core()
    cams = synth.sphere_camera()
    rgb, ns, sig = _render(sphere, core.Rays.cameras(cams), storage=storage)
    o, d = O.camera_rays(cams)
    # arithmetic-only: the oracle reads the same rounded leaves
    ref_r = O.render(oracle_tree(sphere, storage), o, d)
    e_arith = rgb_err(rgb, ref_r)
    # quantisation-inclusive: the oracle reads the FP64 generator values
    ref_q = O.render(O.OracleTree.from_scene(sphere), o, d)
    e_q = rgb_err(rgb, ref_q)
    print(f"{storage}: arithmetic max {e_arith.max():.3e}; vs FP64 values max {e_q.max():.3e} "
          f"p99 {np.quantile(e_q, 0.99):.3e} mean {e_q.mean():.3e}")
    assert e_arith.max() <= TOL32
    assert e_q.max() <= TOL16


@pytest.mark.parametrize("storage,degree", [("f16", 3), ("bf16", 3), ("f16", 1), ("bf16", 1)])
def test_reduced_precision_leaves_degrees_1_and_3(storage, degree):
    """16-bit leaves at degrees 1 and 3 (the benchmark's degree; the sphere
    tests cover degree 2): against the oracle on the same rounded leaves the
    arithmetic alone stays within the FP32 tolerance, and against the FP64
    generator values within the 2e-3 gate."""
    core = _core()
    s = synth.random_tree_scene(5, degree, seed=80 + degree, p_split=0.5, sigma_max=12.0)
    cams = synth.random_sphere_cameras(3, 3.5, 48, 48, seed=81)
    rgb, ns, sig = _render(s, core.Rays.cameras(cams), storage=storage)
    o, d = O.camera_rays(cams)
    e = rgb_err(rgb, O.render(oracle_tree(s, storage), o, d))
    e_q = rgb_err(rgb, O.render(O.OracleTree.from_scene(s), o, d))
    print(f"{storage} degree {degree}: vs rounded leaves max {e.max():.3e}; vs FP64 values max {e_q.max():.3e}")
    assert e.max() <= TOL32
    assert e_q.max() <= TOL16


def test_torus_box_full_size_all_rays():
    """The 800x800 x 8-camera workload as benchmarked, every one of its
    5,120,000 rays against the oracle (colour and segment count), and the
    fused max-weight signal of that frame, accumulated into a zeroed buffer,
    against the oracle's early/late stopping-rule signals for every leaf."""
    core = _core()
    s = synth.torus_box_scene()
    cams = synth.ring_cameras()
    tree = core.Octree.from_scene(s)
    rays = core.Rays.cameras(cams)
    sig = torch.zeros(tree.n_leaves, dtype=torch.float32, device="cuda")
    rgb_t, ns_t = tree.render(rays, signal=sig, nseg=True)
    torch.cuda.synchronize()
    rgb, ns, gsig = rgb_t.cpu().numpy(), ns_t.cpu().numpy(), sig.cpu().numpy().astype(np.float64)
    tree.close()
    T = oracle_tree(s)
    npx = 800 * 800
    lo = np.zeros(s.n_leaves)
    hi = np.zeros(s.n_leaves)
    emax, n_strad, n_same = 0.0, 0, 0
    for j in range(len(cams)):
        # one camera at a time keeps the oracle's per-ray signal records small
        o, d = O.camera_rays(cams, np.full(npx, j, np.int32), np.arange(npx, dtype=np.int32))
        ref = O.render(T, o, d, signal=True)
        sl = slice(j * npx, (j + 1) * npx)
        e = rgb_err(rgb[sl], ref)
        emax = max(emax, float(e.max()))
        n_strad += int(ref["straddle"].sum())
        n_same += int(((ns[sl] == ref["nseg"]) | ref["straddle"]).sum())
        lo = np.maximum(lo, np.minimum(ref["sig_lo"], ref["sig_hi"]))
        hi = np.maximum(hi, np.maximum(ref["sig_lo"], ref["sig_hi"]))
    bad = (gsig < lo - TOL32) | (gsig > hi + TOL32)
    print(f"torus+box all {rgb.shape[0]} rays: max err {emax:.3e}, straddle {n_strad}, segment counts equal "
          f"{n_same / rgb.shape[0]:.6f}; signal: {int((gsig > 0).sum())} leaves > 0, {int(bad.sum())} outside "
          f"[lo, hi] +- 1e-5, max |gpu - hi| {np.abs(gsig - hi).max():.3e}")
    assert emax <= TOL32
    assert n_same / rgb.shape[0] >= 0.999
    assert not bad.any()
    assert np.isfinite(rgb).all() and rgb.min() >= 0.0 and rgb.max() <= 1.0 + 1e-6


def test_stream_read_probe():
    import ctypes as C
    from paper_2307_15333_amd import _lib as L
    lib = L.load()
    buf = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, device="cuda")
    L.check(lib.dot_stream_read(C.c_void_p(buf.data_ptr()), C.c_size_t(1 << 24), C.c_void_p(sink.data_ptr()), None))
    L.check(lib.dot_stream_read(C.c_void_p(buf.data_ptr()), C.c_size_t(100), C.c_void_p(sink.data_ptr()), None))
    torch.cuda.synchronize()
    assert lib.dot_stream_read(C.c_void_p(buf.data_ptr() + 4), C.c_size_t(64), C.c_void_p(sink.data_ptr()),
                               None) == L.DOT_EINVAL
    # the gather probe over the same 16 MiB (2^16 rows of 192 B fit in 12 MiB), small and odd read counts
    L.check(lib.dot_gather_rows(C.c_void_p(buf.data_ptr()), C.c_int64(1 << 16), C.c_int64(1 << 20),
                                C.c_void_p(sink.data_ptr()), None))
    L.check(lib.dot_gather_rows(C.c_void_p(buf.data_ptr()), C.c_int64(1), C.c_int64(5), C.c_void_p(sink.data_ptr()),
                                None))
    torch.cuda.synchronize()
    assert lib.dot_gather_rows(C.c_void_p(buf.data_ptr()), C.c_int64(3), C.c_int64(5), C.c_void_p(sink.data_ptr()),
                               None) == L.DOT_EINVAL
    # the atomic probe: every increment lands (plain and returning), on few and on many counters
    for k in (7, 1 << 16):
        cnt = torch.zeros(k, dtype=torch.int32, device="cuda")
        L.check(lib.dot_atomic_count(C.c_void_p(cnt.data_ptr()), C.c_uint32(k), C.c_int64(300001), 0, None))
        L.check(lib.dot_atomic_count(C.c_void_p(cnt.data_ptr()), C.c_uint32(k), C.c_int64(200000), 1, None))
        torch.cuda.synchronize()
        c = cnt.cpu().numpy().astype(np.int64)
        assert c.sum() == 500001 and (c >= 0).all() and (k > 1000 or (c > 0).all())
