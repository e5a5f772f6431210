"""Serving: one persistent launch over many requests and resident trees.

A request's image must be the same alone and inside any mix (bitwise: the same
per-ray code runs on the same tree and camera), equal to dot_render's image,
and within tolerance of the oracle.  Admission never exceeds the HBM budget.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2307_15333_amd import synth

pytestmark = pytest.mark.gpu


def _mods():
    from paper_2307_15333_amd import core, serve
    return core, serve


@pytest.fixture(scope="module")
def trees():
    core, _ = _mods()
    scenes = [synth.sphere_scene(),
              synth.make_scene(synth.sdf_sphere(0.4, (0.1, -0.1, 0.0)), 5, 2, seed=7),
              synth.random_tree_scene(6, 3, seed=3, p_split=0.4, sigma_max=15.0),
              synth.random_tree_scene(6, 3, seed=4, p_split=0.4, sigma_max=15.0)]
    ts = [core.Octree.from_scene(s, "f16") for s in scenes]
    yield scenes, ts
    for t in ts:
        t.close()


def _req(serve, i, tree, w, h, az, el):
    cam = synth.look_at_camera(az, el, 4.0, w, h)
    return serve.Request(rid=i, tree=tree, cam=cam, width=w, height=h, arrival=0.0)


def test_alone_equals_mix_and_dot_render(trees):
    core, serve = _mods()
    scenes, ts = trees
    srv = serve.Server(ts)
    a = _req(serve, 0, 1, 128, 96, 30.0, 20.0)
    others = [_req(serve, 1, 0, 256, 256, 100.0, -10.0), _req(serve, 2, 2, 200, 120, 210.0, 40.0),
              _req(serve, 3, 3, 64, 64, 300.0, 5.0)]
    for r in [a] + others:
        srv._admit(r, 0.0)
    srv.launch([(a, 0, a.n_tiles)])
    alone = a.out.clone()
    a.out.zero_()
    # the same request split in two, interleaved with three other requests on other trees
    half = a.n_tiles // 2
    srv.launch([(others[0], 0, others[0].n_tiles), (a, half, a.n_tiles - half), (others[1], 0, others[1].n_tiles),
                (a, 0, half), (others[2], 0, others[2].n_tiles)])
    torch.cuda.synchronize()
    assert torch.equal(alone, a.out)
    # dot_render of the same camera
    rays = core.Rays.cameras(np.asarray(a.cam).reshape(1))
    ref = ts[1].render(rays).reshape(96, 128, 3)
    np.testing.assert_allclose(alone.cpu().numpy(), ref.cpu().numpy(), atol=1e-6, rtol=0)
    # the oracle on the same FP16-rounded leaves
    s = scenes[1]
    T = O.OracleTree(s.child, O.round_storage(s.sigma.astype(np.float64), "f16"),
                     O.round_storage(s.sh.astype(np.float64), "f16"), s.degree)
    o, d = O.camera_rays(np.asarray(a.cam).reshape(1))
    r = O.render(T, o, d)
    g = alone.cpu().numpy().reshape(-1, 3).astype(np.float64)
    e = np.minimum(np.abs(g - r["rgb"]).max(1), np.minimum(np.abs(g - r["rgb_early"]).max(1),
                                                          np.abs(g - r["rgb_late"]).max(1)))
    assert e.max() <= 1e-5
    # the other requests match their own dot_render images too
    for q in others:
        ref = ts[q.tree].render(core.Rays.cameras(np.asarray(q.cam).reshape(1))).reshape(q.height, q.width, 3)
        np.testing.assert_allclose(q.out.cpu().numpy(), ref.cpu().numpy(), atol=1e-6, rtol=0)


def test_poisson_load_results_and_latency(trees):
    core, serve = _mods()
    scenes, ts = trees
    reqs = serve.poisson_requests(len(ts), rate=200.0, duration=1.5, seed=4,
                                  resolutions=[(128, 128), (256, 256), (333, 251)])
    check = {}

    def keep(r):
        if r.rid % 7 == 0:
            check[r.rid] = r.out.clone()

    srv = serve.Server(ts, out_budget_bytes=64 << 20, max_tiles=2048)
    st = srv.run(reqs, on_complete=keep)
    print(st)
    assert st["requests"] == len(reqs) and st["rejected"] == 0
    assert st["max_budget_used"] <= st["budget"]
    assert st["p50_ms"] is not None and st["p99_ms"] >= st["p50_ms"]
    # every kept result equals the same request rendered alone
    for r in reqs:
        if r.rid in check:
            rays = core.Rays.cameras(np.asarray(r.cam).reshape(1))
            ref = ts[r.tree].render(rays).reshape(r.height, r.width, 3)
            np.testing.assert_allclose(check[r.rid].cpu().numpy(), ref.cpu().numpy(), atol=1e-6, rtol=0)


def test_admission_budget_and_rejection(trees):
    core, serve = _mods()
    scenes, ts = trees
    big = _req(serve, 0, 0, 512, 512, 10.0, 10.0)            # 3 MiB of output
    small = [_req(serve, i, i % 4, 128, 128, 40.0 * i, 0.0) for i in range(1, 9)]  # 192 KiB each
    srv = serve.Server(ts, out_budget_bytes=1 << 20, max_tiles=256)
    st = srv.run([big] + small)
    assert st["rejected"] == 1 and st["requests"] == 8
    assert st["max_budget_used"] <= 1 << 20


def test_job_validation(trees):
    import ctypes as C
    from paper_2307_15333_amd import _lib as L
    core, serve = _mods()
    scenes, ts = trees
    srv = serve.Server(ts)
    r = _req(serve, 0, 0, 64, 64, 0.0, 0.0)
    srv._admit(r, 0.0)
    with pytest.raises(L.DotError) as e:
        srv.launch([(r, 60, 10)])                 # 64 tiles in the image
    assert e.value.code == L.DOT_EINVAL and "tile range" in str(e.value)
    jobs = (L.dot_render_job * 1)()
    assert srv.lib.dot_render_jobs(jobs, 1, C.c_void_p(srv._workspace(1).data_ptr()), 16, None) == L.DOT_EINVAL


def test_batch_mixing_storage_types():
    """One batch over trees of all four storage types (one launch per type,
    tiles of one image split and interleaved with the others): each image
    equals dot_render's, and a one-tile batch (fewer workgroups than chunks)
    completes too."""
    core, serve = _mods()
    s = synth.sphere_scene()
    ts = [core.Octree.from_scene(s, st) for st in ("f32", "f16", "bf16", "f32")]
    ts[3].quantize_sh(8)                                         # palette leaves
    srv = serve.Server(ts)
    reqs = [_req(serve, i, i, w, h, 70.0 * i, 15.0 - 10.0 * i)
            for i, (w, h) in enumerate(((96, 80), (64, 64), (120, 72), (80, 96)))]
    for r in reqs:
        srv._admit(r, 0.0)
    a, b, c, d = reqs
    ha = a.n_tiles // 2
    srv.launch([(a, ha, a.n_tiles - ha), (b, 0, b.n_tiles), (c, 0, c.n_tiles), (a, 0, ha), (d, 0, d.n_tiles)])
    tiny = _req(serve, 9, 1, 8, 8, 5.0, 5.0)
    srv._admit(tiny, 0.0)
    srv.launch([(tiny, 0, 1)])
    torch.cuda.synchronize()
    for r in reqs + [tiny]:
        ref = ts[r.tree].render(core.Rays.cameras(np.asarray(r.cam).reshape(1))).reshape(r.height, r.width, 3)
        np.testing.assert_allclose(r.out.cpu().numpy(), ref.cpu().numpy(), atol=1e-6, rtol=0)
    for t in ts:
        t.close()
