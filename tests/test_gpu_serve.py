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


def test_launches_carry_several_requests_under_load(trees):
    """Under an offered load beyond what the host issues launches for (small
    images at 60,000 req/s, one launch in flight at a time), each launch
    carries several requests that arrived while the previous one ran, and
    every checked request still equals its image rendered alone."""
    core, serve = _mods()
    scenes, ts = trees
    reqs = serve.poisson_requests(len(ts), rate=60000.0, duration=0.15, seed=14,
                                  resolutions=[(128, 128), (256, 256), (333, 251)])
    check = {}

    def keep(r):
        if r.rid % 11 == 0:
            check[r.rid] = r.out.clone()

    srv = serve.Server(ts, out_budget_bytes=256 << 20, max_tiles=8192, max_inflight=1)
    st = srv.run(reqs, on_complete=keep)
    print({k: st[k] for k in ("requests", "launches", "mean_requests_per_launch", "p50_ms", "p99_ms")})
    assert st["requests"] == len(reqs)
    assert st["mean_requests_per_launch"] >= 4.0
    for r in reqs:
        if r.rid in check:
            ref = ts[r.tree].render(core.Rays.cameras(np.asarray(r.cam).reshape(1))).reshape(r.height, r.width, 3)
            np.testing.assert_allclose(check[r.rid].cpu().numpy(), ref.cpu().numpy(), atol=1e-6, rtol=0)


def _reference_images(core, ts, reqs):
    return {r.rid: ts[r.tree].render(core.Rays.cameras(np.asarray(r.cam).reshape(1))).reshape(r.height, r.width, 3)
            .cpu().numpy() for r in reqs}


def test_persistent_queue_alone_equals_mix(trees):
    """The persistent launch: a request rendered alone, then again while five
    other requests (on the other trees) are queued with it and its own image
    is pushed as two jobs in reverse tile order -- bitwise the same image,
    equal to the batched launch's and within 1e-6 of dot_render's; the other
    requests match dot_render too.  References are rendered before the queue
    opens and results read after it closes (the open launch holds the GPU)."""
    core, serve = _mods()
    scenes, ts = trees
    a = _req(serve, 0, 1, 128, 96, 30.0, 20.0)
    others = [_req(serve, 1 + i, (i % 3) + (i % 3 >= 1), w, h, 50.0 * i, 10.0 - 5.0 * i)
              for i, (w, h) in enumerate(((256, 256), (200, 120), (64, 64), (333, 251), (96, 160)))]
    ref = _reference_images(core, ts, [a] + others)
    srv = serve.Server(ts)
    srv._admit(a, 0.0)
    srv.launch([(a, 0, a.n_tiles)])
    batched = a.out.cpu().numpy()
    alone = torch.zeros((a.height, a.width, 3), device="cuda")
    mixed = torch.zeros((a.height, a.width, 3), device="cuda")
    outs = [torch.zeros((r.height, r.width, 3), device="cuda") for r in others]
    torch.cuda.synchronize()
    q = serve.Queue("f16", max_jobs=32, max_seconds=8.0)
    try:
        q.wait(q.push(ts[a.tree], a.cam, alone, a.width, a.height))
        n = a.n_tiles
        tickets = [q.push(ts[others[0].tree], others[0].cam, outs[0], others[0].width, others[0].height),
                   q.push(ts[a.tree], a.cam, mixed, a.width, a.height, tile_begin=n // 2, tile_count=n - n // 2)]
        for r, o in zip(others[1:], outs[1:]):
            tickets.append(q.push(ts[r.tree], r.cam, o, r.width, r.height))
        tickets.append(q.push(ts[a.tree], a.cam, mixed, a.width, a.height, tile_begin=0, tile_count=n // 2))
        assert all(t is not None for t in tickets)
        for t in tickets:
            q.wait(t)
    finally:
        q.close()
    al, mx = alone.cpu().numpy(), mixed.cpu().numpy()
    assert np.array_equal(al, mx)
    assert np.array_equal(al, batched)
    np.testing.assert_allclose(al, ref[a.rid], atol=1e-6, rtol=0)
    for r, o in zip(others, outs):
        np.testing.assert_allclose(o.cpu().numpy(), ref[r.rid], atol=1e-6, rtol=0)


def test_persistent_results_readable_while_the_launch_runs(trees):
    """A job's image is complete and visible to other device work as soon as
    its completion word says so, while the launch keeps running: each image
    is copied out on a side stream right after its job completes (jobs pushed
    one at a time and in bursts, poisoned outputs first) and equals the image
    dot_render gives."""
    core, serve = _mods()
    scenes, ts = trees
    sizes = ((128, 96), (256, 256), (64, 64), (333, 251), (200, 120), (96, 160), (512, 384), (8, 8))
    reqs = [_req(serve, i, i % 4, w, h, 37.0 * i, 25.0 - 7.0 * i) for i, (w, h) in enumerate(sizes)]
    ref = _reference_images(core, ts, reqs)
    outs = [torch.full((r.height, r.width, 3), -7.0, device="cuda") for r in reqs]
    hosts = [torch.empty((r.height, r.width, 3), pin_memory=True) for r in reqs]
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    q = serve.Queue("f16", max_jobs=32, max_seconds=20.0)

    def read(i):
        with torch.cuda.stream(side):
            hosts[i].copy_(outs[i], non_blocking=True)
        side.synchronize()
        np.testing.assert_allclose(hosts[i].numpy(), ref[reqs[i].rid], atol=1e-6, rtol=0)

    try:
        for i in range(3):                       # one at a time
            r = reqs[i]
            q.wait(q.push(ts[r.tree], r.cam, outs[i], r.width, r.height))
            read(i)
        burst = {}
        for i in range(3, len(reqs)):            # a burst, read as each completes
            r = reqs[i]
            burst[i] = q.push(ts[r.tree], r.cam, outs[i], r.width, r.height)
        import time
        t0 = time.perf_counter()
        while burst:
            assert time.perf_counter() - t0 < 10.0, f"jobs {sorted(burst)} not done"
            for i, tk in list(burst.items()):
                if q.done(tk):
                    read(i)
                    del burst[i]
    finally:
        q.close()


def test_persistent_small_request_overtakes_a_large_one(trees):
    """The feeder gives jobs with few entries left all of them before the room
    goes to larger jobs: an 8x8 request pushed right after a 4096x4096 one
    (262,144 tiles) completes while the large one is still rendering, and both
    images equal dot_render's."""
    import time
    core, serve = _mods()
    scenes, ts = trees
    big = _req(serve, 0, 2, 4096, 4096, 20.0, 10.0)
    tiny = _req(serve, 1, 0, 8, 8, 200.0, -20.0)
    ref = _reference_images(core, ts, [big, tiny])
    out_big = torch.zeros((big.height, big.width, 3), device="cuda")
    out_tiny = torch.zeros((tiny.height, tiny.width, 3), device="cuda")
    torch.cuda.synchronize()
    q = serve.Queue("f16", max_jobs=8, max_seconds=20.0)
    try:
        tb = q.push(ts[big.tree], big.cam, out_big, big.width, big.height)
        tt = q.push(ts[tiny.tree], tiny.cam, out_tiny, tiny.width, tiny.height)
        t0 = time.perf_counter()
        while not q.done(tt):
            assert time.perf_counter() - t0 < 10.0
        t_tiny = time.perf_counter() - t0
        big_done_first = q.done(tb)
        q.wait(tb, timeout=10.0)
    finally:
        q.close()
    print(f"tiny done after {1e3 * t_tiny:.3f} ms (big done by then: {big_done_first})")
    assert not big_done_first
    np.testing.assert_allclose(out_tiny.cpu().numpy(), ref[tiny.rid], atol=1e-6, rtol=0)
    np.testing.assert_allclose(out_big.cpu().numpy(), ref[big.rid], atol=1e-6, rtol=0)


def test_persistent_queue_limits_and_time_limit(trees):
    """A queue refuses a tree of another storage type and a tile range outside
    the image; it reports a full queue (2^19 tiles of unfinished jobs) without
    queuing, and takes the job once the earlier one completed; a launch past
    its time limit ends by itself and the queue then refuses new jobs."""
    import time
    from paper_2307_15333_amd import _lib as L
    core, serve = _mods()
    scenes, ts = trees
    t32 = core.Octree.from_scene(scenes[0], "f32")
    cam = synth.look_at_camera(20.0, 10.0, 4.0, 8192, 4096)
    big = torch.empty((4096, 8192, 3), device="cuda")
    small = torch.empty((8, 8, 3), device="cuda")
    cam8 = synth.look_at_camera(20.0, 10.0, 4.0, 8, 8)
    torch.cuda.synchronize()
    q = serve.Queue("f16", max_jobs=4, max_seconds=8.0)
    try:
        with pytest.raises(L.DotError) as e:
            q.push(t32, cam8, small, 8, 8)
        assert e.value.code == L.DOT_EINVAL
        with pytest.raises(L.DotError) as e:
            q.push(ts[0], cam8, small, 8, 8, tile_begin=1, tile_count=1)
        assert e.value.code == L.DOT_EINVAL
        tb = q.push(ts[0], cam, big, 8192, 4096)          # 2^19 tiles
        assert tb is not None
        busy = q.push(ts[0], cam8, small, 8, 8)
        q.wait(tb)
        ts_ = q.push(ts[0], cam8, small, 8, 8) if busy is None else busy
        assert ts_ is not None
        q.wait(ts_)
        print(f"full queue reported: {busy is None}")
    finally:
        q.close()
    q = serve.Queue("f16", max_jobs=4, max_seconds=0.2)
    try:
        time.sleep(0.6)
        with pytest.raises(L.DotError) as e:
            q.push(ts[0], cam8, small, 8, 8)
        assert e.value.code == L.DOT_EHIP
    finally:
        q.close()
    t32.close()


def test_persistent_server_poisson(trees):
    """The persistent server under Poisson arrivals: every request completes,
    and checked results equal the same requests rendered alone."""
    core, serve = _mods()
    scenes, ts = trees
    reqs = serve.poisson_requests(len(ts), rate=3000.0, duration=0.4, seed=24,
                                  resolutions=[(128, 128), (256, 256), (333, 251)])
    ref = _reference_images(core, ts, [r for r in reqs if r.rid % 9 == 0])
    torch.cuda.synchronize()
    srv = serve.PersistentServer(ts, out_budget_bytes=256 << 20, max_seconds=8.0)
    st = srv.run(reqs, keep_outputs=True)
    print({k: st[k] for k in ("requests", "p50_ms", "p99_ms", "mrays_per_s")})
    assert st["requests"] == len(reqs) and st["rejected"] == 0
    for r in reqs:
        if r.rid in ref:
            np.testing.assert_allclose(r.out.cpu().numpy(), ref[r.rid], atol=1e-6, rtol=0)
