"""Continuous-batching render server over octrees resident in HBM.

Requests (tree, camera, resolution) arrive over time.  Each scheduling
iteration the server

  1. admits arrived requests in arrival order while the HBM budget for output
     images and the slot limit allow (a request larger than the whole budget is
     rejected),
  2. packs the next tiles of the admitted requests, oldest first, into one
     batch of at most `max_tiles` 8x8 tiles -- a large image is split over
     several batches, so requests that arrive while others run join the next
     batch instead of waiting for whole images --
  3. launches the batch as ONE persistent kernel (`dot_render_jobs`) over all
     resident trees, keeping up to `max_inflight` batches queued on the stream
     so the device never idles while the host packs the next one,
  4. retires launches whose completion event has fired; a request completes
     with the launch that rendered its last tile, and frees its slot and budget.

While work is queued or running the loop polls (no sleep), so completions and
arrivals are seen within one event query; when idle it sleeps until `spin_s`
before the next arrival.

Latency = completion time - arrival time (host clock, event-polled).  Each
launch is bracketed by two timing events; the union of those intervals over
the run gives the fraction of the wall time the GPU spent in launches.  The
image a request receives is independent of the batch it was packed into: every
pixel runs the same per-ray code on the same tree and camera.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import time
from collections import deque

import numpy as np
import torch

from . import _lib as L
from . import core


@dataclasses.dataclass
class Request:
    rid: int
    tree: int
    cam: np.ndarray          # one camera record (synth.CAMERA_DTYPE)
    width: int
    height: int
    arrival: float           # seconds from the start of the run
    bg: tuple = (1.0, 1.0, 1.0)
    t_stop: float = 1e-4
    # runtime state
    n_tiles: int = 0
    next_tile: int = 0
    out: torch.Tensor | None = None
    cam_dev: torch.Tensor | None = None
    admitted: float = -1.0
    done: float = -1.0
    ticket: int = -1
    arena_off: int = -1

    @property
    def rays(self):
        return self.width * self.height

    @property
    def out_bytes(self):
        return self.rays * 12


class Server:
    def __init__(self, trees, out_budget_bytes=2 << 30, max_active=64, max_tiles=65536, max_inflight=2,
                 device="cuda", spin_s=3e-4, streams=1):
        self.trees = trees
        self.lib = L.load()
        self.device = torch.device(device)
        self.budget = int(out_budget_bytes)
        self.max_active = int(max_active)
        self.max_tiles = int(max_tiles)
        self.max_inflight = int(max_inflight)
        self.spin_s = float(spin_s)
        self.used = 0
        self.max_used = 0
        # launches go round-robin over `streams` streams (default priority), each
        # with its own job-table workspace, so a batch can start while the
        # previous one drains; with one stream they run back to back
        self.streams = [torch.cuda.current_stream(self.device)] if streams <= 1 else \
            [torch.cuda.Stream(self.device) for _ in range(streams)]
        self.ws = [None] * len(self.streams)
        self.ws_bytes = [0] * len(self.streams)
        self._next_stream = 0

    def _workspace(self, n_jobs, k=0):
        need = int(self.lib.dot_render_jobs_workspace(n_jobs))
        if need > self.ws_bytes[k]:
            with torch.cuda.stream(self.streams[k]):
                self.ws[k] = torch.empty(need * 2, dtype=torch.uint8, device=self.device)
            self.ws_bytes[k] = need * 2
        return self.ws[k]

    def _admit(self, req, now):
        req.n_tiles = ((req.width + 7) // 8) * ((req.height + 7) // 8)
        req.next_tile = 0
        req.out = torch.empty((req.height, req.width, 3), dtype=torch.float32, device=self.device)
        raw = np.ascontiguousarray(np.asarray(req.cam).reshape(1)).view(np.uint8)
        # pinned source, so the upload is queued on the stream without a host wait
        req.cam_dev = torch.from_numpy(raw.copy()).pin_memory().to(self.device, non_blocking=True)
        req.admitted = now
        self.used += req.out_bytes
        self.max_used = max(self.max_used, self.used)

    def launch(self, batch, k=0):
        """batch: list of (request, tile_begin, tile_count) -> one persistent launch on stream k."""
        n = len(batch)
        jobs = (L.dot_render_job * n)()
        for i, (r, b, c) in enumerate(batch):
            j = jobs[i]
            j.tree = self.trees[r.tree].handle
            j.cam = r.cam_dev.data_ptr()
            j.rgb_out = r.out.data_ptr()
            j.width, j.height = r.width, r.height
            j.tile_begin, j.tile_count = b, c
            for a in range(3):
                j.bg[a] = float(r.bg[a])
            j.t_stop = float(r.t_stop)
        ws = self._workspace(n, k)
        if self.streams[k] != torch.cuda.current_stream(self.device):
            # the cameras were uploaded on the current stream at admission
            self.streams[k].wait_stream(torch.cuda.current_stream(self.device))
        L.check(self.lib.dot_render_jobs(jobs, n, C.c_void_p(ws.data_ptr()), C.c_size_t(self.ws_bytes[k]),
                                         C.c_void_p(self.streams[k].cuda_stream)))

    def run(self, requests, duration=None, warmup=0.0, keep_outputs=False, on_complete=None):
        """Serve `requests` (sorted by arrival) in real time.  Returns stats over
        the requests that arrived at or after `warmup` seconds."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting, active, inflight = deque(), [], deque()
        completed, rejected = [], []
        t0 = time.perf_counter()
        launches = 0
        tiles_launched = 0
        reqs_launched = 0
        spans = []
        torch.cuda.synchronize(self.device)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        while pending or waiting or active or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # 1. admission by slots and HBM budget, in arrival order
            while waiting and len(active) < self.max_active:
                r = waiting[0]
                if r.out_bytes > self.budget:
                    rejected.append(waiting.popleft())
                    continue
                if self.used + r.out_bytes > self.budget:
                    break
                self._admit(waiting.popleft(), now)
                active.append(r)
            # 2-3. pack the next batch and launch it
            if len(inflight) < self.max_inflight:
                batch, finishing, room = [], [], self.max_tiles
                for r in active:
                    if room == 0:
                        break
                    left = r.n_tiles - r.next_tile
                    if left == 0:
                        continue
                    c = min(left, room)
                    batch.append((r, r.next_tile, c))
                    r.next_tile += c
                    room -= c
                    if r.next_tile == r.n_tiles:
                        finishing.append(r)
                if batch:
                    k = self._next_stream
                    self._next_stream = (k + 1) % len(self.streams)
                    st = self.streams[k]
                    ev0 = torch.cuda.Event(enable_timing=True)
                    ev0.record(st)
                    self.launch(batch, k)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(st)
                    inflight.append((ev, finishing, ev0))
                    launches += 1
                    tiles_launched += self.max_tiles - room
                    reqs_launched += len(batch)
                    continue
            # 4. retire finished launches in order
            progressed = False
            while inflight and inflight[0][0].query():
                ev, fin, ev0 = inflight.popleft()
                spans.append((ref.elapsed_time(ev0), ref.elapsed_time(ev)))
                t_done = time.perf_counter() - t0
                for r in fin:
                    r.done = t_done
                    active.remove(r)
                    self.used -= r.out_bytes
                    if on_complete is not None:
                        on_complete(r)
                    if not keep_outputs:
                        r.out = None
                        r.cam_dev = None
                    completed.append(r)
                progressed = True
            if not progressed and pending and not waiting and not active and not inflight:
                # idle: sleep until shortly before the next arrival (a sleep
                # overshoots by tens of microseconds), then poll
                dt = pending[0].arrival - (time.perf_counter() - t0)
                if dt > self.spin_s:
                    time.sleep(min(dt - self.spin_s, 0.002))
            # with work queued or running the loop polls without sleeping, so a
            # completion or an arrival is seen within one event query
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # GPU busy time: the union of the launches' [start, end] intervals
        busy_ms, end_ms = 0.0, -1.0
        for a, b in sorted(spans):
            if b > end_ms:
                busy_ms += b - max(a, end_ms)
                end_ms = b
        meas = [r for r in completed if r.arrival >= warmup]
        lat = np.array([r.done - r.arrival for r in meas]) * 1e3
        rays = sum(r.rays for r in meas)
        span = (max(r.done for r in meas) - min(r.arrival for r in meas)) if meas else 0.0
        return {
            "requests": len(meas), "rejected": len(rejected), "launches": launches,
            "p50_ms": float(np.percentile(lat, 50)) if meas else None,
            "p99_ms": float(np.percentile(lat, 99)) if meas else None,
            "mean_ms": float(lat.mean()) if meas else None,
            "max_ms": float(lat.max()) if meas else None,
            "mrays_per_s": rays / span / 1e6 if span > 0 else None,
            "req_per_s": len(meas) / span if span > 0 else None,
            "wall_s": wall, "mean_tiles_per_launch": tiles_launched / max(launches, 1),
            "mean_requests_per_launch": reqs_launched / max(launches, 1),
            "gpu_busy_frac": busy_ms / 1e3 / wall if wall > 0 else None,
            "max_budget_used": self.max_used, "budget": self.budget,
        }


class Queue:
    """The persistent serving launch (dot_serve_*): one launch on its own stream
    renders the jobs pushed while it runs."""

    def __init__(self, storage="f16", max_jobs=1024, max_seconds=3600.0, device="cuda"):
        self.lib = L.load()
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)      # occupied by the launch until close()
        h = C.c_void_p()
        st = {**L.STORAGE, "pal16": L.DOT_PAL16}[storage]
        L.check(self.lib.dot_serve_open(st, int(max_jobs), float(max_seconds),
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def push(self, tree, cam, rgb_out, width, height, tile_begin=0, tile_count=None, bg=(1.0, 1.0, 1.0),
             t_stop=1e-4):
        """Queue the tiles [tile_begin, tile_begin + tile_count) of one image; returns the
        job's ticket, or None when the queue is full."""
        n_tiles = ((width + 7) // 8) * ((height + 7) // 8)
        j = L.dot_serve_job()
        j.tree = tree.handle
        j.cam = L.dot_camera.from_buffer_copy(np.ascontiguousarray(np.asarray(cam).reshape(1)).tobytes())
        j.rgb_out = rgb_out.data_ptr()
        j.width, j.height = int(width), int(height)
        j.tile_begin = int(tile_begin)
        j.tile_count = int(n_tiles - tile_begin if tile_count is None else tile_count)
        for a in range(3):
            j.bg[a] = float(bg[a])
        j.t_stop = float(t_stop)
        t = C.c_int64()
        rc = self.lib.dot_serve_push(self.h, C.byref(j), C.byref(t))
        if rc == L.DOT_EBUSY:
            return None
        L.check(rc)
        return t.value

    def done(self, ticket):
        rc = self.lib.dot_serve_done(self.h, C.c_int64(ticket))
        if rc < 0:
            L.check(rc)
        return rc == 1

    def wait(self, ticket, timeout=5.0):
        t0 = time.perf_counter()
        while not self.done(ticket):
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"serving job {ticket} not done after {timeout} s")

    def close(self):
        if self.h:
            L.check(self.lib.dot_serve_close(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PersistentServer:
    """Continuous batching through the persistent launch: each admitted request
    is pushed at once as one job (its whole image) into the running launch, so
    its tiles are taken by waves that are free now, beside the tiles of the
    requests already on the device; admission (slots, HBM budget for outputs)
    and latency as in Server."""

    def __init__(self, trees, out_budget_bytes=2 << 30, max_active=64, device="cuda", storage="f16",
                 max_seconds=3600.0):
        self.trees = trees
        self.device = torch.device(device)
        self.budget = int(out_budget_bytes)
        self.max_active = int(max_active)
        self.storage = storage
        self.max_seconds = float(max_seconds)
        self.used = 0

    def run(self, requests, warmup=0.0, keep_outputs=False, on_complete=None):
        """Serve `requests` in real time.  Outputs come from an arena of the
        HBM budget, allocated before the launch and reused once a request has
        completed (no allocator call while the launch holds the GPU); with
        keep_outputs each request gets its own buffer instead, allocated before
        the launch starts and valid after run() returns.  on_complete(r) is called on the host when r completes:
        r.out is then whole and may be read by device work on a stream other than the queue's (a copy into host
        memory, say; work on the queue's stream would wait for the launch to end).  With the arena that work must
        have finished when on_complete returns, since r's region is then reused."""
        arena = None if keep_outputs else torch.empty(self.budget, dtype=torch.uint8, device=self.device)
        if keep_outputs:
            # every request's own output, allocated before the launch holds the GPU
            for r in requests:
                r.out = torch.empty((r.height, r.width, 3), dtype=torch.float32, device=self.device)
        free = [(0, self.budget)]          # free byte ranges of the arena, sorted

        def alloc(nbytes):
            nbytes = (nbytes + 255) & ~255
            for i, (a, n) in enumerate(free):
                if n >= nbytes:
                    free[i:i + 1] = [(a + nbytes, n - nbytes)] if n > nbytes else []
                    return a
            return None

        def release(a, nbytes):
            nbytes = (nbytes + 255) & ~255
            free.append((a, nbytes))
            free.sort()
            merged = []
            for x, n in free:
                if merged and merged[-1][0] + merged[-1][1] == x:
                    merged[-1] = (merged[-1][0], merged[-1][1] + n)
                else:
                    merged.append((x, n))
            free[:] = merged

        q = Queue(self.storage, max_jobs=max(2 * self.max_active, 16), max_seconds=self.max_seconds,
                  device=self.device)
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting, active, completed, rejected = deque(), [], [], []
        t0 = time.perf_counter()
        try:
            while pending or waiting or active:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                while waiting and len(active) < self.max_active:
                    r = waiting[0]
                    if r.out_bytes > self.budget:
                        rejected.append(waiting.popleft())
                        continue
                    if self.used + r.out_bytes > self.budget:
                        break
                    r.n_tiles = ((r.width + 7) // 8) * ((r.height + 7) // 8)
                    if not keep_outputs:
                        off = alloc(r.out_bytes)
                        if off is None:     # fragmented arena: wait for a completion
                            break
                        r.arena_off = off
                        r.out = arena[off:off + r.out_bytes].view(torch.float32).view(r.height, r.width, 3)
                    tk = q.push(self.trees[r.tree], r.cam, r.out, r.width, r.height, bg=r.bg, t_stop=r.t_stop)
                    if tk is None:          # queue full: retry after a completion
                        if not keep_outputs:
                            release(r.arena_off, r.out_bytes)
                        r.out = None
                        break
                    r.ticket = tk
                    r.admitted = now
                    self.used += r.out_bytes
                    active.append(waiting.popleft())
                still = []
                for r in active:
                    if q.done(r.ticket):
                        r.done = time.perf_counter() - t0
                        self.used -= r.out_bytes
                        if on_complete is not None:
                            on_complete(r)
                        if not keep_outputs:
                            release(r.arena_off, r.out_bytes)
                            r.out = None
                        completed.append(r)
                    else:
                        still.append(r)
                active = still
                if not active and not waiting and pending:
                    dt = pending[0].arrival - (time.perf_counter() - t0)
                    if dt > 3e-4:
                        time.sleep(min(dt - 3e-4, 0.002))
        finally:
            q.close()
        wall = time.perf_counter() - t0
        meas = [r for r in completed if r.arrival >= warmup]
        lat = np.array([r.done - r.arrival for r in meas]) * 1e3
        rays = sum(r.rays for r in meas)
        span = (max(r.done for r in meas) - min(r.arrival for r in meas)) if meas else 0.0
        return {
            "requests": len(meas), "rejected": len(rejected), "launches": 1,
            "p50_ms": float(np.percentile(lat, 50)) if meas else None,
            "p99_ms": float(np.percentile(lat, 99)) if meas else None,
            "mean_ms": float(lat.mean()) if meas else None,
            "max_ms": float(lat.max()) if meas else None,
            "mrays_per_s": rays / span / 1e6 if span > 0 else None,
            "req_per_s": len(meas) / span if span > 0 else None,
            "wall_s": wall, "mean_tiles_per_launch": float(sum(r.n_tiles for r in completed)),
            "mean_requests_per_launch": float(len(completed)), "gpu_busy_frac": None,
            "budget": self.budget,
        }


RESOLUTIONS = [(128, 128), (256, 256), (512, 512), (800, 800), (1920, 1080)]


def poisson_requests(n_trees, rate, duration, seed, resolutions=RESOLUTIONS, radius=4.0):
    """Poisson arrivals at `rate` req/s over `duration` s; resolution, tree and a
    camera on the radius-4 sphere drawn uniformly (seeded)."""
    from . import synth
    rng = np.random.default_rng(seed)
    t, out, i = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        w, h = resolutions[rng.integers(len(resolutions))]
        v = rng.normal(size=3)
        v *= radius / np.linalg.norm(v)
        cam = synth._camera_at(v, w, h, 40.0)
        out.append(Request(rid=i, tree=int(rng.integers(n_trees)), cam=cam, width=w, height=h, arrival=t))
        i += 1
    return out
