"""Benchmark of the octree volume renderer on one MI355X.

Step = one forward render (Eq. 1-2) of the 800x800 x 8-camera workload
(torus+box SDF octree of depth 9, 3.54M leaves, SH degree 3, FP32 leaves),
inputs resident in HBM.  The JSON line also carries the roofline of the render
kernel (compulsory bytes: every distinct leaf the frame composites fetched
once; beside them the counter traffic of the same launch kind and the two
measured ceilings, streaming reads and random 192-byte row gathers), the same
frame with the fused max-weight signal (its buffer cleared in every step), the
FP64 CPU oracle as a baseline, and the other measured forms of the hot path
(FP16/BF16/palette leaves, the device-wide atomic rate that bounds the
training forward's counting, the differentiable training step, Alg. 1
epochs, refinement, serving latency on the persistent launch and on
relaunches).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s render & train step (FP32 vs FP16 leaves); p50/p99 served latency"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "render_fwd_torus_box_traffic.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2307_15333_amd", "csrc")
    for f in ("dot_device.h", "render.hip", "dot_internal.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    rec = None
    for line in open(PROFILE_TRAFFIC):
        if line.startswith("TRAFFIC_JSON "):
            rec = json.loads(line[len("TRAFFIC_JSON "):])
    if not rec or rec.get("kernel_src_sha") != kernel_source_hash():
        return None
    return rec


def time_kernel(fn, reps, torch, warmup=3):
    """Median duration of `fn` (the launches it queues on the current stream)
    over `reps` calls, each bracketed by HIP events recorded on that stream,
    after `warmup` untimed calls."""
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(s)
        fn()
        b.record(s)
    ev[-1][1].synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev])) / 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-terrain", action="store_true", help="skip the 19M-leaf terrain precision run")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--alg1-epochs", type=int, default=4, help="epochs of the end-to-end training loop (0: skip)")
    ap.add_argument("--only", choices=["train", "alg1", "refine", "serve", "serve_sweep", "terrain", "palette",
                                       "ablation"],
                    help="run one secondary measurement alone and print its JSON (for profiling it)")
    ap.add_argument("--profile-copy", nargs="?", const="plain", choices=["plain", "fused"],
                    help="run one 1 GiB device copy and four renders of the timed kind (counter runs)")
    ap.add_argument("--profile-dtypes", action="store_true",
                    help="render the benchmark frame once per leaf storage (FP32, FP16, BF16) for counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the renderer would shard by rays "
              "with the tree replicated and one all-reduce (max) of the signal, which is not run here.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2307_15333_amd import core, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    if args.only in ("train", "terrain"):
        fn = {"train": train_step, "terrain": terrain_precision}[args.only]
        print(json.dumps(fn(torch, core, synth, args)), flush=True)
        return
    scene = synth.torus_box_scene()
    cams = synth.ring_cameras()
    log(f"torus+box scene: {scene.n_leaves} leaves, {scene.n_internal} internal ({time.time() - t0:.1f}s)")
    if args.only:
        fn = {"alg1": lambda: alg1_loop(torch, core, synth, scene, args),
              "palette": lambda: palette_render(torch, core, scene, core.Rays.cameras(cams), None, args),
              "ablation": lambda: ablation(torch, core, synth, scene, cams, args),
              "refine": lambda: refine_pass(torch, core, synth, scene),
              "serve": lambda: serving(torch, core, synth, scene, args),
              "serve_sweep": lambda: serving_sweep(torch, core, synth, scene, args)}[args.only]
        print(json.dumps(fn()), flush=True)
        return
    tree = core.Octree.from_scene(scene, "f32")
    rays = core.Rays.cameras(cams)
    n_rays = rays.n_rays
    signal = torch.zeros(tree.n_leaves, dtype=torch.float32, device=dev)
    rgb = torch.empty((n_rays, 3), dtype=torch.float32, device=dev)
    import ctypes as C
    from paper_2307_15333_amd import _lib as L
    opts = core.render_opts(t_stop=1e-4)
    lib = L.load()

    def step():
        # the timed step: the plain render of the 8 views (no signal)
        L.check(lib.dot_render(tree.handle, C.byref(rays.struct), C.byref(opts), C.c_void_p(rgb.data_ptr()),
                               None, None, core._stream()))

    def fused_step():
        # render with the fused max-weight signal into a signal buffer cleared first
        signal.zero_()
        L.check(lib.dot_render(tree.handle, C.byref(rays.struct), C.byref(opts), C.c_void_p(rgb.data_ptr()),
                               None, C.c_void_p(signal.data_ptr()), core._stream()))

    if args.profile_dtypes:
        for st in ("f32", "f16", "bf16"):
            t = tree if st == "f32" else core.Octree.from_scene(scene, st)
            for _ in range(3):
                L.check(lib.dot_render(t.handle, C.byref(rays.struct), C.byref(opts), C.c_void_p(rgb.data_ptr()),
                                       None, None, core._stream()))
            torch.cuda.synchronize()
            if t is not tree:
                t.close()
        log("profile-dtypes: three plain renders per storage type done")
        return
    if args.profile_copy:
        # counter calibration: a copy of known size, then the launch kind bench.py
        # times (one warm-up render, then three timed-like renders back to back)
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        for _ in range(4):
            fused_step() if args.profile_copy == "fused" else step()
        torch.cuda.synchronize()
        log(f"profile-copy: one 1 GiB copy and four {args.profile_copy} renders done")
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms = elapsed / args.steps * 1e3
    value = n_rays / (elapsed / args.steps) / 1e6
    log(f"render fp32 (plain): {ms:.3f} ms/step, {value:.1f} Mrays/s")

    # ---- roofline of the render kernel ----
    stats = tree.render_stats(rays)
    K = (scene.degree + 1) ** 2
    row_bytes = 4 + 3 * K * 4
    leaf_bytes = stats["segments"] * 4 + stats["sh_fetches"] * 3 * K * 4
    kt = time_kernel(step, max(20, args.steps), torch)
    other = stats["index_reads"] * 4 + n_rays * 12
    # compulsory bytes: every distinct leaf the frame composites, fetched once
    # (a leaf with a positive signal received a positive weight, hence an SH
    # fetch), plus the image written once
    fused_step()
    n_touched = int((signal > 0).sum().item())
    compulsory = n_touched * row_bytes + n_rays * 12
    achieved = compulsory / kt / 1e9
    traffic = read_traffic()
    tb = None if traffic is None else traffic["hbm_bytes_per_launch"]
    achievable = stream_read_gbps(torch, L, lib)
    gather = gather_rows_gbps(torch, L, lib)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tb,
                "kernel": "render_fwd_kernel<F32,deg3> (plain render, no signal)", "kernel_ms": round(kt * 1e3, 4),
                "per_unit": f"{row_bytes} B per distinct leaf composited (4 B sigma + {3 * K * 4} B SH, fetched "
                            "once) + 12 B rgb per ray",
                "units_per_launch": {"distinct_leaves_composited": n_touched, "rays": n_rays},
                "compulsory_bytes_per_launch": int(compulsory),
                "traffic_over_compulsory": None if tb is None else round(tb / compulsory, 2),
                "traffic_GBps": None if tb is None else round(tb / kt / 1e9, 1),
                "traffic_note": "FETCH_SIZE x read scale + WRITE_SIZE x write scale per plain render launch "
                                "(rocprofv3, same launch kind as timed); FETCH_SIZE counts Infinity-Cache hits "
                                "as well as HBM reads, so it bounds HBM traffic from above",
                "cache_inclusive_leaf_bytes_per_launch": int(leaf_bytes),
                "cache_inclusive_leaf_GBps": round(leaf_bytes / kt / 1e9, 1),
                "cache_inclusive_per_unit": "4 B sigma per segment + 192 B SH per segment with sigma*delta > 0 "
                                            "(what the lanes request; caches serve most of it)",
                "cache_inclusive_units": {"segments": stats["segments"], "sh_fetches": stats["sh_fetches"]},
                "other_bytes_per_launch": {"child_and_link_reads": stats["index_reads"] * 4, "rgb": n_rays * 12,
                                           "total": int(other)},
                "achievable_read_GBps": round(achievable, 1),
                "achievable_gather_rows": gather,
                "traffic_over_gather_ceiling": None if tb is None else round(tb / kt / 1e9 / gather["line_GBps"], 3)}
    log(f"render kernel {kt * 1e3:.3f} ms; compulsory {achieved:.1f} GB/s ({achieved / HBM_PEAK_GBS:.1%} of HBM "
        f"peak); cache-inclusive leaf bytes {leaf_bytes / kt / 1e9:.1f} GB/s; segments/ray "
        f"{stats['segments'] / n_rays:.2f}")
    fused = fused_signal_forms(torch, tree, rays, signal, rgb, fused_step, args)

    extra = {}
    if not args.no_extra:
        extra = measure_extra(torch, core, synth, scene, cams, tree, args)
    tree.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene, cams)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded SDF octree, random SH; stands in for NeRF-synthetic 800x800 views)",
        "config": {"workload": "torus+box SDF octree, depth 9, %d leaves, SH degree 3, FP32 leaves, "
                               "8 cameras x 800x800 on the radius-4 sphere, white bg, t_stop 1e-4, plain "
                               "render" % scene.n_leaves,
                   "rays_per_step": n_rays, "parallelism": "single GPU",
                   "signal": "none in the timed step; the fused max-weight signal is timed separately "
                             "(fused_signal), its buffer cleared inside every step"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fused_signal": fused,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def stream_read_gbps(torch, L, lib):
    """Achievable HBM read bandwidth: dot_stream_read over a 4 GiB buffer."""
    import ctypes as C
    from paper_2307_15333_amd import core
    nbytes = 4 << 30
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")

    def fn():
        L.check(lib.dot_stream_read(C.c_void_p(buf.data_ptr()), C.c_size_t(nbytes), C.c_void_p(sink.data_ptr()),
                                    core._stream()))

    kt = time_kernel(fn, 10, torch)
    del buf
    gbps = nbytes / kt / 1e9
    log(f"stream read: {gbps:.1f} GB/s achievable ({gbps / HBM_PEAK_GBS:.1%} of the 8 TB/s peak)")
    return gbps


def gather_rows_gbps(torch, L, lib):
    """The leaf-fetch pattern without its dependences: dot_gather_rows reads
    16M random 192-byte rows (each lane a whole row) of a 3 GiB buffer; a row
    at a 192-byte stride spans exactly two 128-byte lines."""
    import ctypes as C
    from paper_2307_15333_amd import core
    n_rows = 1 << 24
    buf = torch.empty(n_rows * 192, dtype=torch.uint8, device="cuda")
    buf.fill_(1)
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    threads = cus * 4 * 256
    reads = max(1, n_rows // threads) * threads          # what the launch reads (a whole number per thread)

    def fn():
        L.check(lib.dot_gather_rows(C.c_void_p(buf.data_ptr()), C.c_int64(n_rows), C.c_int64(n_rows),
                                    C.c_void_p(sink.data_ptr()), core._stream()))

    kt = time_kernel(fn, 10, torch)
    del buf
    out = {"rows_per_s_G": round(reads / kt / 1e9, 2), "row_GBps": round(reads * 192 / kt / 1e9, 1),
           "line_GBps": round(reads * 256 / kt / 1e9, 1),
           "note": "random 192 B rows, one per lane per step, over 3 GiB (2 lines of 128 B per row)"}
    log(f"gather rows: {out['rows_per_s_G']} G rows/s = {out['row_GBps']} GB/s of row bytes, "
        f"{out['line_GBps']} GB/s of lines")
    return out


def fused_signal_forms(torch, tree, rays, signal, rgb, fused_step, args):
    """The render with the fused max-weight signal (Sec. 3.1) on the benchmark
    frame.  Each timed step clears the signal buffer and renders into it, so
    every launch issues the atomics of a fresh signal; the clear alone is timed
    beside it.  The steady state -- the same frame rendered again into a filled
    buffer, where the max filter skips every atomic -- is reported as a
    labelled extra only."""
    import ctypes as C
    from paper_2307_15333_amd import _lib as L, core
    reps = max(20, args.steps)
    kt = time_kernel(fused_step, reps, torch)
    fill = time_kernel(signal.zero_, reps, torch)
    op = core.render_opts()

    def steady():
        L.check(tree.lib.dot_render(tree.handle, C.byref(rays.struct), C.byref(op), C.c_void_p(rgb.data_ptr()),
                                    None, C.c_void_p(signal.data_ptr()), core._stream()))

    ks = time_kernel(steady, reps, torch)
    out = {"ms_per_step": round(kt * 1e3, 4), "mrays": round(rays.n_rays / kt / 1e6, 1),
           "signal_clear_ms": round(fill * 1e3, 4), "render_ms": round((kt - fill) * 1e3, 4),
           "steady_state_filled_buffer_ms": round(ks * 1e3, 4),
           "note": "step = clear the [L] signal + render with fused max-weight signal; steady state = the same "
                   "frame into an already filled buffer (no atomics pass the filter), not a workload"}
    log(f"render fp32 + fused signal (cleared each step): {kt * 1e3:.3f} ms ({rays.n_rays / kt / 1e6:.1f} Mrays/s; "
        f"clear {fill * 1e3:.3f} ms); steady state into a filled buffer {ks * 1e3:.3f} ms")
    return out


def render_times(torch, core, tree, rays, args):
    """(plain render time, render-with-fused-signal time incl. the signal clear) of one tree."""
    import ctypes as C
    from paper_2307_15333_amd import _lib as L
    sig = torch.zeros(tree.n_leaves, dtype=torch.float32, device="cuda")
    rgb = torch.empty((rays.n_rays, 3), dtype=torch.float32, device="cuda")
    op = core.render_opts()

    def plain():
        L.check(tree.lib.dot_render(tree.handle, C.byref(rays.struct), C.byref(op), C.c_void_p(rgb.data_ptr()),
                                    None, None, core._stream()))

    def fused():
        sig.zero_()
        L.check(tree.lib.dot_render(tree.handle, C.byref(rays.struct), C.byref(op), C.c_void_p(rgb.data_ptr()),
                                    None, C.c_void_p(sig.data_ptr()), core._stream()))

    reps = max(20, args.steps)
    return time_kernel(plain, reps, torch), time_kernel(fused, reps, torch), rgb


def measure_extra(torch, core, synth, scene, cams, tree_f32, args):
    """FP16/BF16 leaves on the same workload, plain and with the fused signal
    (cleared each step), then the other forms of the path."""
    res = {}
    rays = core.Rays.cameras(cams)
    base = None
    for storage in ("f32", "f16", "bf16"):
        tree = tree_f32 if storage == "f32" else core.Octree.from_scene(scene, storage)
        kp, kf, _ = render_times(torch, core, tree, rays, args)
        mp, mf = rays.n_rays / kp / 1e6, rays.n_rays / kf / 1e6
        if storage == "f32":
            base = (mp, mf)
        res[f"render_{storage}_mrays"] = round(mp, 1)
        res[f"render_{storage}_fused_signal_mrays"] = round(mf, 1)
        if storage != "f32":
            res[f"render_{storage}_speedup_vs_f32"] = round(mp / base[0], 3)
            res[f"render_{storage}_fused_signal_speedup_vs_f32"] = round(mf / base[1], 3)
            tree.close()
        log(f"render {storage}: plain {kp * 1e3:.3f} ms ({mp:.1f} Mrays/s), with fused signal {kf * 1e3:.3f} ms "
            f"({mf:.1f} Mrays/s)")
    res.update(palette_render(torch, core, scene, rays, base, args))
    res["atomic_count"] = atomic_count_rate(torch)
    res.update(train_step(torch, core, synth, args))
    if args.alg1_epochs > 0:
        res.update(alg1_loop(torch, core, synth, scene, args))
    res.update(refine_pass(torch, core, synth, scene))
    res.update(serving(torch, core, synth, scene, args))
    if not args.no_terrain:
        res.update(terrain_precision(torch, core, synth, args))
    return res


def atomic_count_rate(torch):
    """Device-wide 32-bit atomic increments per second (dot_atomic_count): 2^24
    of them spread by a hash over 2^20 counters, over the 3,536,632 leaves of
    the torus+box tree and over the 8,632 of the sphere tree, each with the
    returned values unused and used (the training forward's counts and its
    slot reservations)."""
    import ctypes as C
    from paper_2307_15333_amd import _lib as L, core
    lib = L.load()
    n = 1 << 24
    out = {}
    for label, k in (("2^20 counters", 1 << 20), ("3536632 counters", 3536632), ("8632 counters", 8632)):
        cnt = torch.zeros(k, dtype=torch.int32, device="cuda")
        r = {}
        for ret in (0, 1):
            def fn():
                L.check(lib.dot_atomic_count(C.c_void_p(cnt.data_ptr()), C.c_uint32(k), C.c_int64(n), ret,
                                             core._stream()))
            r["returning" if ret else "plain"] = round(n / time_kernel(fn, 10, torch) / 1e9, 2)
        out[label] = r
    log(f"atomic increments, G/s (plain / returning): " +
        ", ".join(f"{lb} {v['plain']} / {v['returning']}" for lb, v in out.items()))
    out["unit"] = "G atomic increments/s"
    return out


def palette_render(torch, core, scene, rays, base_mrays, args):
    """The torus+box octree compressed by the median-cut palette (2^16 FP16 rows, FP16 sigma,
    uint16 index per leaf): build time, render Mrays/s (plain and with the fused
    signal cleared each step), and the image difference against the FP32 tree."""
    ref_tree = core.Octree.from_scene(scene, "f32")
    ref = ref_tree.render(rays)
    ref_tree.close()
    tree = core.Octree.from_scene(scene, "f32")
    torch.cuda.synchronize()
    t = time.perf_counter()
    tree.quantize_sh(16)
    torch.cuda.synchronize()
    t_q = time.perf_counter() - t
    kp, kf, rgb = render_times(torch, core, tree, rays, args)
    mp, mf = rays.n_rays / kp / 1e6, rays.n_rays / kf / 1e6
    mse = float(((rgb - ref) ** 2).mean())
    psnr = 10 * np.log10(1.0 / mse) if mse > 0 else float("inf")
    tree.close()
    sp = mp / base_mrays[0] if base_mrays else None
    sf = mf / base_mrays[1] if base_mrays else None
    log(f"render pal16 (median cut, 2^16 rows): quantize {t_q * 1e3:.0f} ms, plain {kp * 1e3:.3f} ms ({mp:.1f} "
        f"Mrays/s, x{sp if sp is None else round(sp, 2)} FP32), fused signal {mf:.1f} Mrays/s, PSNR vs FP32 tree "
        f"{psnr:.1f} dB")
    return {"render_pal16_mrays": round(mp, 1), "render_pal16_speedup_vs_f32": None if sp is None else round(sp, 3),
            "render_pal16_fused_signal_mrays": round(mf, 1),
            "render_pal16_fused_signal_speedup_vs_f32": None if sf is None else round(sf, 3),
            "pal16_quantize_ms": round(t_q * 1e3, 1), "pal16_psnr_vs_f32_db": round(psnr, 2)}


def ablation(torch, core, synth, scene, cams, args):
    """Synthetic stand-in for the paper's signal and fusion ablations (Tab. 3,
    App. C.1) on the torus+box octree: targets are the generator tree's renders
    from 100 random 400x400 views (16M rays per epoch); training starts from
    SH + N(0, 0.1^2); 4 epochs of 2^20-ray batches with RMSProp and a
    refinement after epochs 2 and 4.  Prune-only runs (gamma = 0) compare the
    max and sum of ray weights (Q) with the density (Pr_sigma, its tau chosen
    to prune about as many leaves as Q-max does first); fusion against
    re-initialised new leaves uses pruning and sampling (gamma = 1 %).  For each
    run: leaves, FP32 render Mrays/s of the 8 benchmark cameras, and PSNR of
    those images against the generator tree."""
    from paper_2307_15333_amd import train as TR
    views = synth.random_sphere_cameras(100, 4.0, 400, 400, seed=31)
    gt = core.Octree.from_scene(scene)
    target = gt.render(core.Rays.cameras(views))
    bench_rays = core.Rays.cameras(cams)
    ref = gt.render(bench_rays)
    gt.close()
    start = synth.perturb_sh(scene, 0.1, seed=32)

    def run(name, **kw):
        tree = core.Octree.from_scene(start)
        cfg = TR.TrainConfig(interval=2, batch_rays=1 << 20, max_depth=10, seed=33, **kw)
        tr = TR.Trainer(tree, views, target, cfg)
        hist = tr.train(epochs=4)
        rgb = tree.render(bench_rays)
        mse = float(((rgb - ref) ** 2).mean())
        sig = torch.zeros(tree.n_leaves, dtype=torch.float32, device="cuda")
        kt = time_kernel(lambda: tree.render(bench_rays, signal=sig), 5, torch)
        out = {"leaves": tree.n_leaves, "leaves_after_first_refine": hist[1]["leaves"],
               "render_mrays": round(bench_rays.n_rays / kt / 1e6, 1),
               "psnr_db": round(float(10 * np.log10(1.0 / mse)), 2) if mse > 0 else None,
               "loss_first_last": [float(hist[0]["losses"].mean()), float(hist[-1]["losses"].mean())]}
        tree.close()
        log(f"ablation {name}: {out}")
        return out

    res = {"ablation_start_leaves": scene.n_leaves}
    res["prune_q_max"] = run("prune Q max (tau 1e-3)", signal="max", tau=1e-3, gamma=0.0)
    res["prune_q_sum"] = run("prune Q sum (tau 1)", signal="sum", tau=1.0, gamma=0.0)
    # Pr_sigma: the density threshold that prunes about as many leaves as Q-max's first pruning
    target_removed = scene.n_leaves - res["prune_q_max"]["leaves_after_first_refine"]
    tau_s, best = None, None
    for t in (0.1, 1.0, 3.0, 10.0, 20.0, 30.0, 40.0, 50.0):
        tree = core.Octree.from_scene(start)
        st = tree.refine(tree.sigma_signal(), prune_tau=t, sample_frac=0.0, max_depth=10)
        tree.close()
        gap = abs((st["leaves_before"] - st["leaves_after"]) - target_removed)
        if best is None or gap < best:
            tau_s, best = t, gap
    res["prune_sigma"] = run(f"prune sigma (tau {tau_s})", signal="sigma", tau=tau_s, gamma=0.0)
    res["prune_sigma"]["tau"] = tau_s
    res["fusion"] = run("prune + sample, fused", signal="max", tau=1e-3, gamma=0.01)
    res["reinit"] = run("prune + sample, re-initialised", signal="max", tau=1e-3, gamma=0.01, reinit=True)
    return res


def refine_pass(torch, core, synth, scene):
    """Refinement of the torus+box octree: max-weight signal over 100 random 800x800 views,
    then top 5% subdivided (max depth 10) and signal <= 1e-3 pruned."""
    tree = core.Octree.from_scene(scene, "f32")
    views = synth.sphere_views(100)
    sig = torch.zeros(tree.n_leaves, dtype=torch.float32, device="cuda")
    n_rays = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    for j in range(0, 100, 10):
        r = core.Rays.cameras(views[j:j + 10])
        tree.accumulate_signal(r, sig)
        n_rays += r.n_rays
    torch.cuda.synchronize()
    t_sig = time.perf_counter() - t
    t = time.perf_counter()
    st = tree.refine(sig, prune_tau=1e-3, sample_frac=0.05, max_depth=10)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t
    tree.close()
    log(f"refine: signal over {n_rays / 1e6:.0f}M rays {t_sig * 1e3:.1f} ms ({n_rays / t_sig / 1e6:.0f} Mrays/s); "
        f"refine {t_ref * 1e3:.1f} ms {st}")
    return {"signal_100views_ms": round(t_sig * 1e3, 2), "signal_mrays": round(n_rays / t_sig / 1e6, 1),
            "refine_ms": round(t_ref * 1e3, 2), "refine_stats": st}


def serving_trees(core, synth, c2_scene):
    """The four resident FP16 trees of the serving workload: two 8.6k-leaf
    spheres (the second re-seeded), the 3.5M-leaf torus+box tree and a copy of
    it with re-drawn SH."""
    import dataclasses
    s1a = synth.sphere_scene()
    s1b = synth.make_scene(synth.sdf_sphere(0.5), 5, 2, seed=40)
    rng = np.random.default_rng(41)
    sh_b = c2_scene.sh32.copy()
    sh_b[:, :, 1:] = (rng.standard_normal(sh_b[:, :, 1:].shape, dtype=np.float32) * np.float32(0.1))
    s2b = dataclasses.replace(c2_scene, sh32=sh_b)
    return [core.Octree.from_scene(x, "f16") for x in (s1a, s1b, c2_scene, s2b)]


def serve_once(serve, trees, rate, seconds, seed=4, warm=2.0, persistent=False, **kw):
    reqs = serve.poisson_requests(4, rate=rate, duration=warm + seconds, seed=seed)
    if persistent:
        srv = serve.PersistentServer(trees, out_budget_bytes=2 << 30)
    else:
        srv = serve.Server(trees, out_budget_bytes=2 << 30, max_tiles=65536, **kw)
    st = srv.run(reqs, warmup=warm)
    offered = sum(r.rays for r in reqs if r.arrival >= warm) / seconds / 1e6
    out = {"rate_req_s": rate, "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
           "mean_ms": round(st["mean_ms"], 3), "mrays": round(st["mrays_per_s"], 1),
           "offered_mrays": round(offered, 1), "req_per_s": round(st["req_per_s"], 1),
           "requests": st["requests"], "launches": st["launches"],
           "requests_per_launch": round(st["mean_requests_per_launch"], 2),
           "tiles_per_launch": round(st["mean_tiles_per_launch"], 1),
           "gpu_busy_frac": None if st["gpu_busy_frac"] is None else round(st["gpu_busy_frac"], 3),
           "seconds": seconds, "mode": "persistent launch" if persistent else "launch per batch"}
    log(f"serving at {rate} req/s: {out}")
    return out


def serving(torch, core, synth, c2_scene, args):
    """Serving: four resident FP16 trees (two 8.6k-leaf spheres, two 3.5M-leaf torus+box trees),
    Poisson arrivals at 200 req/s, resolutions uniform over {128^2, 256^2, 512^2,
    800^2, 1920x1080}; latency percentiles after a warm-up.  Config 5's numbers
    come from the persistent launch (each admitted request's tiles join the
    running launch at once); the same arrivals served by one launch per
    scheduling iteration are reported beside them."""
    from paper_2307_15333_amd import serve
    trees = serving_trees(core, synth, c2_scene)
    st = serve_once(serve, trees, 200.0, args.serve_seconds, persistent=True)
    rl = serve_once(serve, trees, 200.0, args.serve_seconds)
    for t in trees:
        t.close()
    return {"serve_p50_ms": st["p50_ms"], "serve_p99_ms": st["p99_ms"], "serve_mean_ms": st["mean_ms"],
            "serve_mrays": st["mrays"], "serve_offered_mrays": st["offered_mrays"], "serve_req_per_s": st["req_per_s"],
            "serve_requests": st["requests"], "serve_seconds": args.serve_seconds,
            "serve_mode": "one persistent launch (dot_serve_*): requests join it as they are admitted",
            "serve_relaunch_p50_ms": rl["p50_ms"], "serve_relaunch_p99_ms": rl["p99_ms"],
            "serve_relaunch_mrays": rl["mrays"], "serve_relaunch_launches": rl["launches"],
            "serve_relaunch_requests_per_launch": rl["requests_per_launch"],
            "serve_relaunch_gpu_busy_frac": rl["gpu_busy_frac"]}


def serving_sweep(torch, core, synth, c2_scene, args):
    """The serving workload at offered loads from 200 req/s to beyond
    saturation (about 611k rays per request, so 6000 req/s offers ~3.7 Grays/s):
    per load p50/p99 latency, throughput, requests and tiles per launch, and the
    fraction of the wall time the GPU spent in launches; launches on one stream
    (back to back) and round-robin over two streams (a batch can start while
    the previous one drains); and the persistent launch that takes each
    request's job as soon as it is admitted (dot_serve_*)."""
    from paper_2307_15333_amd import serve
    trees = serving_trees(core, synth, c2_scene)
    rates = (200.0, 1000.0, 3000.0, 6000.0)
    out = {"sweep": [dict(serve_once(serve, trees, r, args.serve_seconds, streams=k), streams=k)
                     for k in (1, 2) for r in rates]}
    out["persistent"] = [serve_once(serve, trees, r, args.serve_seconds, persistent=True) for r in rates]
    for t in trees:
        t.close()
    return out


def terrain_precision(torch, core, synth, args):
    """Precision on the 19M-leaf terrain + ellipsoids octree, 4 views at 1920x1080,
    leaves stored in FP32 / FP16 / BF16; throughput per dtype and error against
    the FP64 oracle on the generator values (4096 sampled rays)."""
    from oracle import oracle as O
    t0 = time.time()
    s = synth.terrain_scene()
    cams = synth.terrain_cameras()
    log(f"terrain scene: {s.n_leaves} leaves ({time.time() - t0:.0f}s)")
    rays = core.Rays.cameras(cams)
    rng = np.random.default_rng(0)
    idx = rng.choice(rays.n_rays, 4096, replace=False)
    npx = 1920 * 1080
    o, d = O.camera_rays(cams, (idx // npx).astype(np.int32), (idx % npx).astype(np.int32))
    ref = O.render(O.OracleTree.from_scene(s), o, d)
    out = {"terrain_leaves": s.n_leaves}
    for storage in ("f32", "f16", "bf16"):
        tree = core.Octree.from_scene(s, storage)
        rgb = tree.render(rays)
        kt = time_kernel(lambda: tree.render(rays), 3, torch)
        g = rgb.cpu().numpy()[idx].astype(np.float64)
        e = np.minimum(np.abs(g - ref["rgb"]).max(1),
                       np.minimum(np.abs(g - ref["rgb_early"]).max(1), np.abs(g - ref["rgb_late"]).max(1)))
        out[f"terrain_{storage}"] = {"mrays": round(rays.n_rays / kt / 1e6, 1), "err_max": float(e.max()),
                                     "err_p99": float(np.quantile(e, 0.99)), "err_mean": float(e.mean())}
        log(f"terrain {storage}: {rays.n_rays / kt / 1e6:.0f} Mrays/s, err max {e.max():.2e} "
            f"p99 {np.quantile(e, 0.99):.2e} mean {e.mean():.2e}")
        tree.close()
    return out


def _train_setup(torch, core, synth):
    gt = synth.sphere_scene()
    start = synth.perturb_sh(gt, 0.05, seed=3)
    views = synth.training_views(100)
    gt_tree = core.Octree.from_scene(gt)
    target = gt_tree.render(core.Rays.cameras(views))           # [100*64*64, 3]
    gt_tree.close()
    return core.Octree.from_scene(start), views, target


def train_step(torch, core, synth, args):
    """The differentiable training step: forward, MSE, hand-written backward,
    Adam, over 2^18 random rays of 100 64x64 views of the 8.6k-leaf sphere
    octree (SH perturbed by N(0, 0.05^2)).  Config 4's number is the step
    through the autograd Function (DotRender, MSELoss, loss.backward(), with
    Adam applied inside the adjoint by FusedAdam).  Beside it: the training
    driver's step (adjoint and Adam fused, no autograd), and the autograd step
    with dense gradients returned to autograd, PyTorch's MSE and a separate
    Adam kernel.  Each route: 3 warm-up steps, then the median of 5 runs of 20
    steps (each run's mean step time is logged)."""
    from paper_2307_15333_amd import train as TR
    B = 1 << 18
    steps = 20
    W = H = 64

    def timed(step_fn, n_warm=3, reps=5):
        # the median over `reps` runs of `steps` consecutive steps: the routes
        # through autograd are bound by the host, where one stray pause (a
        # garbage collection, another process) moves a 20-step mean by tens
        # of microseconds; training continues from one run to the next
        for k in range(n_warm):
            step_fn()
        torch.cuda.synchronize()
        per, first, last = [], None, None
        for _ in range(reps):
            losses = []
            t = time.perf_counter()
            for _ in range(steps):
                losses.append(step_fn())
            torch.cuda.synchronize()
            per.append((time.perf_counter() - t) / steps)
            first = float(losses[0]) if first is None else first
            last = float(losses[-1])
        return float(np.median(per)), first, last, [round(x * 1e3, 3) for x in per]

    # the training driver
    tree, views, target = _train_setup(torch, core, synth)
    tr = TR.Trainer(tree, views, target, TR.TrainConfig(optimizer="adam", batch_rays=B, refine=False, seed=3))
    idx = tr.permutation()[:B]
    dd, d0, d1, dreps = timed(lambda: tr.step(idx))
    tree.close()
    log(f"train step (training driver): {dd * 1e3:.3f} ms, {B / dd / 1e6:.1f} Mrays/s, loss {d0:.3e} -> {d1:.3e} "
        f"(runs {dreps} ms)")

    def autograd_step_fn(dense):
        tree, views, target = _train_setup(torch, core, synth)
        _, cams_raw = core.Rays._cams_tensor(views, "cuda")
        sigma, sh = tree.plane_views()
        p_sig, p_sh = sigma.detach().requires_grad_(), sh.detach().requires_grad_()     # alias the planes
        opt = None if dense else core.FusedAdam(tree)
        state = tree.adam_state() if dense else None
        st = {"ws": None, "k": 0, "pb": None}

        def step():
            # the batch's buffers are kept from one step to the next, as the training driver keeps them
            cam, pix, ids, st["ws"] = core.pixel_batch(idx, W, H, len(views), st["ws"], out=st["pb"])
            st["pb"] = (cam, pix, ids)
            rays = core.Rays.pixels_device(cams_raw, len(views), cam, pix)
            if dense:
                rgb = core.render_autograd(tree, p_sig, p_sh, rays)
                loss = torch.nn.functional.mse_loss(rgb, target[ids])
                p_sig.grad = p_sh.grad = None
                loss.backward()
                st["k"] += 1
                tree.adam_step(p_sig.grad, p_sh.grad, state, st["k"])
            else:
                rgb = core.render_autograd(tree, p_sig, p_sh, rays, optimizer=opt)
                loss = core.mse_loss_autograd(rgb, target, ids)
                loss.backward()
            return loss.detach()

        return tree, step

    tree, fn = autograd_step_fn(False)
    da, a0, a1, areps = timed(fn)
    tree.close()
    log(f"train step (autograd Function, MSELoss, Adam in the adjoint): {da * 1e3:.3f} ms, {B / da / 1e6:.1f} "
        f"Mrays/s, loss {a0:.3e} -> {a1:.3e} (runs {areps} ms)")
    tree, fn = autograd_step_fn(True)
    dn, n0, n1, nreps = timed(fn)
    tree.close()
    log(f"train step (autograd Function, dense gradients, torch MSE, dot_adam_step): {dn * 1e3:.3f} ms, "
        f"{B / dn / 1e6:.1f} Mrays/s, loss {n0:.3e} -> {n1:.3e} (runs {nreps} ms)")
    return {"train_step_ms": round(da * 1e3, 3), "train_step_mrays": round(B / da / 1e6, 1),
            "train_rays_per_step": B, "train_loss_first_last": [a0, a1], "train_step_runs_ms": areps,
            "train_step_note": "config 4 through the autograd Function (DotRender + MSELoss + loss.backward(), "
                               "Adam applied inside the adjoint)",
            "train_driver_step_ms": round(dd * 1e3, 3), "train_driver_step_mrays": round(B / dd / 1e6, 1),
            "train_driver_loss_first_last": [d0, d1], "train_driver_step_runs_ms": dreps,
            "train_autograd_over_driver": round(da / dd, 3),
            "train_step_autograd_dense_ms": round(dn * 1e3, 3),
            "train_step_autograd_dense_mrays": round(B / dn / 1e6, 1),
            "train_autograd_dense_loss_first_last": [n0, n1]}


def alg1_loop(torch, core, synth, scene, args):
    """Alg. 1 end to end on the torus+box octree: 100 random 800x800 views of
    the generator scene as targets (64M rays per epoch), training copy with SH
    perturbed by N(0, 0.05^2); epochs of 2^20-ray batches, RMSProp (lr 0.1 /
    0.01), refinement every 2nd epoch from the fused max-weight signal (prune
    <= 1e-3, top 1% subdivided up to depth 10)."""
    from paper_2307_15333_amd import train as TR
    views = synth.sphere_views(100)
    gt = core.Octree.from_scene(scene)
    W, H = int(views[0]["width"]), int(views[0]["height"])
    target = torch.empty((len(views) * W * H, 3), dtype=torch.float32, device="cuda")
    for j in range(0, len(views), 10):
        target[j * W * H:(j + 10) * W * H] = gt.render(core.Rays.cameras(views[j:j + 10]))
    gt.close()
    tree = core.Octree.from_scene(synth.perturb_sh(scene, 0.05, seed=3))
    cfg = TR.TrainConfig(interval=2, batch_rays=1 << 20, tau=1e-3, gamma=0.01, max_depth=10, seed=1)
    tr = TR.Trainer(tree, views, target, cfg)
    epochs = []
    for e in range(args.alg1_epochs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = tr.run_epoch()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        rec = {"epoch": r["epoch"], "ms": round(dt * 1e3, 1), "mrays": round(tr.n_rays / dt / 1e6, 1),
               "loss_mean": float(r["losses"].mean()), "leaves": r["leaves"]}
        if "refine" in r:
            rec["refine"] = r["refine"]
        epochs.append(rec)
        log(f"alg1 epoch {rec['epoch']}: {rec['ms']:.0f} ms ({rec['mrays']:.0f} Mrays/s), loss {rec['loss_mean']:.3e},"
            f" leaves {rec['leaves']}{' refined' if 'refine' in r else ''}")
    tree.close()
    plain = [x["ms"] for x in epochs if "refine" not in x]
    return {"alg1_rays_per_epoch": tr.n_rays, "alg1_batch": cfg.batch_rays, "alg1_epochs": epochs,
            "alg1_epoch_ms": min(plain) if plain else None,
            "alg1_train_mrays": round(tr.n_rays / (min(plain) / 1e3) / 1e6, 1) if plain else None}


def cpu_baseline(scene, cams):
    """The FP64 oracle, as it stands, on the host cores: all 8 cameras of the
    workload (the same 5.12M rays the GPU step renders); render calls only."""
    from oracle import oracle as O
    T = O.OracleTree.from_scene(scene, sigma=scene.sigma.astype(np.float64))
    return _cpu_result(T, cams)


def _cpu_result(T, cams):
    from oracle import oracle as O
    total = 0.0
    n = 0
    for j in range(len(cams)):
        ci = np.full(800 * 800, j, np.int32)
        pi = np.arange(800 * 800, dtype=np.int32)
        o, d = O.camera_rays(cams, ci, pi)
        t1 = time.perf_counter()
        O.render(T, o, d)
        total += time.perf_counter() - t1
        n += o.shape[0]
    v = n / total / 1e6
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    log(f"cpu oracle: {n} rays in {total:.2f}s = {v:.3f} Mrays/s on {O.num_threads()} threads ({model})")
    return {"value": round(v, 4), "unit": "Mrays/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"all {n} rays of the 8 800x800 views (render calls only, FP64, OpenMP, "
                      f"{O.num_threads()} threads of {os.cpu_count()} CPUs, {model})"}


if __name__ == "__main__":
    main()
