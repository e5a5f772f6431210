"""Python face of libdot: trees, ray batches and the autograd function.

Argument marshalling only: every step of rendering, differentiation,
refinement and optimisation runs in the HIP kernels behind the C ABI.  PyTorch
provides device memory (through the allocator hook) and streams.
"""
from __future__ import annotations

import ctypes as C
import functools

import numpy as np
import torch

from . import _lib as L

_NP_CAMERA = np.dtype([("c2w", np.float32, (12,)), ("fx", np.float32), ("fy", np.float32),
                       ("cx", np.float32), ("cy", np.float32), ("width", np.int32), ("height", np.int32)])
assert _NP_CAMERA.itemsize == C.sizeof(L.dot_camera)


# the current stream's handle without building a torch.cuda.Stream object (a
# few microseconds a call, several calls a training step)
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)
_cur_device = getattr(torch._C, "_cuda_getDevice", None)


def _stream():
    if _raw_stream is not None and _cur_device is not None:
        return C.c_void_p(_raw_stream(_cur_device()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class TorchAllocator:
    """Device allocations for the library served by torch's caching allocator."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.blocks = {}
        self._cb_alloc = L.ALLOC_FN(self._alloc)
        self._cb_free = L.FREE_FN(self._free)
        self.struct = L.dot_allocator(self._cb_alloc, self._cb_free, None)

    def _alloc(self, nbytes, ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.blocks[p] = t
        return p

    def _free(self, p, ctx):
        self.blocks.pop(p, None)

    def tensor(self, ptr, nbytes):
        base = self.blocks[ptr]
        return base[:nbytes]


class Rays:
    """A ray batch: all pixels of cameras, a (camera, pixel) list, or explicit rays."""

    def __init__(self, struct, keep, n_rays, shape=None):
        self.struct = struct
        self._keep = keep
        self.n_rays = int(n_rays)
        self.shape = shape

    @staticmethod
    def _cams_tensor(cams, device):
        cams = np.ascontiguousarray(np.asarray(cams).astype(_NP_CAMERA, copy=False))
        raw = torch.from_numpy(cams.view(np.uint8).copy()).to(device)
        return cams, raw

    @classmethod
    def cameras(cls, cams, device="cuda"):
        cams, raw = cls._cams_tensor(cams, device)
        W, H = int(cams[0]["width"]), int(cams[0]["height"])
        if not all(int(c["width"]) == W and int(c["height"]) == H for c in cams):
            raise ValueError("all cameras of a CAMERAS batch must share width and height")
        s = L.dot_rays(kind=L.DOT_RAYS_CAMERAS, n_cams=len(cams), cams=raw.data_ptr(), width=W, height=H)
        return cls(s, [raw], len(cams) * W * H, (len(cams), H, W))

    @classmethod
    def pixels(cls, cams, cam_idx, pix_idx, device="cuda"):
        cams, raw = cls._cams_tensor(cams, device)
        ci = torch.as_tensor(np.asarray(cam_idx, np.int32)).to(device)
        pi = torch.as_tensor(np.asarray(pix_idx, np.int32)).to(device)
        n = ci.shape[0]
        s = L.dot_rays(kind=L.DOT_RAYS_PIXELS, n_cams=len(cams), cams=raw.data_ptr(), n_rays=n,
                       cam_idx=ci.data_ptr(), pix_idx=pi.data_ptr())
        return cls(s, [raw, ci, pi], n)

    @classmethod
    def pixels_device(cls, cams_raw, n_cams, cam_idx, pix_idx):
        """(camera, pixel) list from tensors already on the device."""
        n = cam_idx.shape[0]
        s = L.dot_rays(kind=L.DOT_RAYS_PIXELS, n_cams=n_cams, cams=cams_raw.data_ptr(), n_rays=n,
                       cam_idx=cam_idx.data_ptr(), pix_idx=pix_idx.data_ptr())
        return cls(s, [cams_raw, cam_idx, pix_idx], n)

    @classmethod
    def explicit(cls, origins, dirs, device="cuda"):
        o = torch.as_tensor(np.asarray(origins, np.float32)).to(device).contiguous()
        d = torch.as_tensor(np.asarray(dirs, np.float32)).to(device).contiguous()
        n = o.shape[0]
        s = L.dot_rays(kind=L.DOT_RAYS_EXPLICIT, n_rays=n, origins=o.data_ptr(), dirs=d.data_ptr())
        return cls(s, [o, d], n)


def render_opts(bg=(1.0, 1.0, 1.0), t_stop=1e-4, signal_mode="max"):
    """A dot_render_opts struct of the caller's own (free to modify)."""
    o = _opts(bg, t_stop, signal_mode)
    return type(o).from_buffer_copy(o)


def _opts(bg=(1.0, 1.0, 1.0), t_stop=1e-4, signal_mode="max"):
    # the binding's calls share one struct per option set: the library only
    # reads it (const pointer) and nothing here writes it
    if not (isinstance(bg, tuple) and len(bg) == 3):
        bg = np.broadcast_to(np.asarray(bg, np.float32), (3,))
    return _render_opts(tuple(float(x) for x in bg), float(t_stop), signal_mode)


@functools.lru_cache(maxsize=64)
def _render_opts(bg, t_stop, signal_mode):
    o = L.dot_render_opts()
    for a in range(3):
        o.bg[a] = bg[a]
    o.t_stop = t_stop
    o.signal_mode = {"max": L.DOT_SIGNAL_MAX, "sum": L.DOT_SIGNAL_SUM}[signal_mode]
    return o


class Octree:
    """A device-resident octree (handle of the C ABI)."""

    def __init__(self, child, sigma, sh, degree, storage="f32", bbox_min=(-1.0, -1.0, -1.0),
                 bbox_size=2.0, device="cuda"):
        self.lib = L.load()
        self.device = torch.device(device)
        self.alloc = TorchAllocator(self.device)
        child = np.ascontiguousarray(child, np.int32).reshape(-1, 8)
        sigma = np.ascontiguousarray(sigma, np.float32)
        K = (degree + 1) ** 2
        sh = np.ascontiguousarray(sh, np.float32).reshape(-1, 3, K)
        desc = L.dot_tree_desc(n_internal=child.shape[0], n_leaves=sigma.shape[0], sh_degree=degree,
                               child=child.ctypes.data, sigma=sigma.ctypes.data, sh=sh.ctypes.data,
                               bbox_size=float(bbox_size))
        for a in range(3):
            desc.bbox_min[a] = float(bbox_min[a])
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.dot_build(C.byref(desc), L.STORAGE[storage], C.byref(self.alloc.struct),
                                       _stream(), C.byref(h)))
        self.handle = h
        self.degree = int(degree)
        self.K = K

    @classmethod
    def from_scene(cls, scene, storage="f32", device="cuda"):
        return cls(scene.child, scene.sigma, scene.sh, scene.degree, storage, scene.bbox_min,
                   scene.bbox_size, device)

    def close(self):
        if getattr(self, "handle", None):
            L.check(self.lib.dot_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- introspection ----
    def info(self):
        i = L.dot_tree_info_t()
        L.check(self.lib.dot_tree_info(self.handle, C.byref(i)))
        return i

    @property
    def n_leaves(self):
        return int(self.info().n_leaves)

    @property
    def n_internal(self):
        return int(self.info().n_internal)

    @property
    def storage(self):
        return L.STORAGE_NAME[int(self.info().storage)]

    def plane_views(self):
        """(sigma [L], sh [L,3,K]) torch views aliasing the device planes."""
        i = self.info()
        Ln = int(i.n_leaves)
        es = 4 if i.storage == L.DOT_F32 else 2
        dt = {L.DOT_F32: torch.float32, L.DOT_F16: torch.float16, L.DOT_BF16: torch.bfloat16}[int(i.storage)]
        sig = self.alloc.tensor(i.sigma, Ln * es).view(dt)
        sh = self.alloc.tensor(i.sh, Ln * int(i.sh_stride) * es).view(dt).view(Ln, int(i.sh_stride))
        sh = sh[:, :3 * self.K].unflatten(1, (3, self.K))
        return sig, sh

    # ---- the C ABI calls ----
    def render(self, rays, bg=(1.0, 1.0, 1.0), t_stop=1e-4, nseg=False, signal=None, signal_mode="max"):
        rgb = torch.empty((rays.n_rays, 3), dtype=torch.float32, device=self.device)
        ns = torch.empty(rays.n_rays, dtype=torch.int32, device=self.device) if nseg else None
        op = _opts(bg, t_stop, signal_mode)
        L.check(self.lib.dot_render(self.handle, C.byref(rays.struct), C.byref(op), _ptr(rgb), _ptr(ns),
                                    _ptr(signal), _stream()))
        return (rgb, ns) if nseg else rgb

    def render_train(self, rays, bg=(1.0, 1.0, 1.0), t_stop=1e-4, signal=None, signal_mode="max", leaf_count=None,
                     records=None, out=None):
        """Training forward: (rgb, nseg, leaf_count) -- leaf_count ([2, L]: recorded and other segments per
        leaf) feeds the adjoint's buckets; `records` (uint8 device buffer of records_bytes(n) bytes, or None)
        receives the segments the adjoint replays.  `out` = (rgb, nseg) of a previous call of the same size is
        written again instead of allocating."""
        if out is not None and out[0].shape[0] == rays.n_rays:
            rgb, ns = out
        else:
            rgb = torch.empty((rays.n_rays, 3), dtype=torch.float32, device=self.device)
            ns = torch.empty(rays.n_rays, dtype=torch.int32, device=self.device)
        if leaf_count is None or leaf_count.numel() < 2 * self.n_leaves:
            leaf_count = torch.empty((2, self.n_leaves), dtype=torch.int32, device=self.device)
        op = _opts(bg, t_stop, signal_mode)
        L.check(self.lib.dot_render_train(self.handle, C.byref(rays.struct), C.byref(op), _ptr(rgb), _ptr(ns),
                                          _ptr(signal), _ptr(leaf_count), _ptr(records),
                                          C.c_size_t(records.numel() if records is not None else 0), _stream()))
        return rgb, ns, leaf_count

    def _take_records(self, n_rays, max_segments):
        """A segment-records buffer for a training forward of n_rays rays with
        room for max_segments per ray: the tree's kept buffer when it is free,
        else a new one (an earlier forward's records still wait for their
        backward)."""
        need = self.records_bytes(n_rays, max_segments)
        if getattr(self, "_rec_busy", False):
            return torch.empty(need, dtype=torch.uint8, device=self.device)
        buf = getattr(self, "_rec_buf", None)
        if buf is None or buf.numel() < need or buf.numel() > 2 * need:
            buf = self._rec_buf = torch.empty(need, dtype=torch.uint8, device=self.device)
        self._rec_busy = True
        return buf[:need]

    def _release_records(self, rec):
        buf = getattr(self, "_rec_buf", None)
        if rec is not None and buf is not None and rec.data_ptr() == buf.data_ptr():
            self._rec_busy = False

    @staticmethod
    @functools.lru_cache(maxsize=64)
    def records_bytes(n_rays, max_segments=96):
        return int(L.load().dot_render_train_records_bytes(int(n_rays), int(max_segments)))

    def accumulate_signal(self, rays, signal, bg=(1.0, 1.0, 1.0), t_stop=1e-4, signal_mode="max"):
        op = _opts(bg, t_stop, signal_mode)
        L.check(self.lib.dot_accumulate_signal(self.handle, C.byref(rays.struct), C.byref(op), _ptr(signal),
                                               _stream()))
        return signal

    def backward(self, rays, rgb, nseg, grad_rgb, grad_sigma, grad_sh, bg=(1.0, 1.0, 1.0), t_stop=1e-4,
                 leaf_count=None, records=None):
        op = _opts(bg, t_stop)
        L.check(self.lib.dot_render_backward(self.handle, C.byref(rays.struct), C.byref(op), _ptr(rgb),
                                             _ptr(nseg), _ptr(grad_rgb), _ptr(grad_sigma), _ptr(grad_sh),
                                             _ptr(leaf_count), _ptr(records),
                                             C.c_size_t(records.numel() if records is not None else 0), _stream()))

    def backward_atomic(self, rays, rgb, nseg, grad_rgb, grad_sigma, grad_sh, bg=(1.0, 1.0, 1.0), t_stop=1e-4):
        """The re-traversal adjoint with per-leaf sums across each wavefront before FP32 atomics (no scratch,
        no synchronisation); accumulates into grad_sigma [L] and grad_sh [L, 3, K]."""
        op = _opts(bg, t_stop)
        L.check(self.lib.dot_render_backward_atomic(self.handle, C.byref(rays.struct), C.byref(op), _ptr(rgb),
                                                    _ptr(nseg), _ptr(grad_rgb), _ptr(grad_sigma), _ptr(grad_sh),
                                                    _stream()))

    def render_stats(self, rays, bg=(1.0, 1.0, 1.0), t_stop=1e-4):
        op = _opts(bg, t_stop)
        out = (C.c_int64 * 4)()
        L.check(self.lib.dot_render_stats(self.handle, C.byref(rays.struct), C.byref(op), out, _stream()))
        return dict(rays=out[0], segments=out[1], sh_fetches=out[2], index_reads=out[3])

    def refine(self, signal, prune_tau=1e-3, sample_frac=0.05, max_depth=10, prune_le=True,
               recursive=False, reinit=False):
        p = L.dot_refine_params(prune_tau=float(prune_tau), sample_frac=float(sample_frac),
                                prune_le=int(bool(prune_le)), max_depth=int(max_depth),
                                recursive=int(bool(recursive)), reinit=int(bool(reinit)))
        st = L.dot_refine_stats()
        L.check(self.lib.dot_refine(self.handle, _ptr(signal), C.byref(p), C.byref(st), _stream()))
        return dict(leaves_before=st.leaves_before, leaves_after=st.leaves_after,
                    internal_after=st.internal_after, merged=st.merged, subdivided=st.subdivided)

    def adam_step(self, grad_sigma, grad_sh, state, step, lr_sigma=0.1, lr_sh=0.01, beta1=0.9,
                  beta2=0.999, eps=1e-8):
        p = L.dot_adam_params(lr_sigma=lr_sigma, lr_sh=lr_sh, beta1=beta1, beta2=beta2, eps=eps, step=int(step))
        L.check(self.lib.dot_adam_step(self.handle, _ptr(grad_sigma), _ptr(grad_sh), _ptr(state["m_sigma"]),
                                       _ptr(state["v_sigma"]), _ptr(state["m_sh"]), _ptr(state["v_sh"]),
                                       C.byref(p), _stream()))

    def adam_state(self):
        Ln = self.n_leaves
        z = lambda *s: torch.zeros(s, dtype=torch.float32, device=self.device)
        return dict(m_sigma=z(Ln), v_sigma=z(Ln), m_sh=z(Ln, 3, self.K), v_sh=z(Ln, 3, self.K))

    def rmsprop_step(self, grad_sigma, grad_sh, state, lr_sigma=0.1, lr_sh=0.01, alpha=0.99, eps=1e-8):
        p = L.dot_rmsprop_params(lr_sigma=lr_sigma, lr_sh=lr_sh, alpha=alpha, eps=eps)
        L.check(self.lib.dot_rmsprop_step(self.handle, _ptr(grad_sigma), _ptr(grad_sh), _ptr(state["v_sigma"]),
                                          _ptr(state["v_sh"]), C.byref(p), _stream()))

    def backward_rmsprop(self, rays, rgb, nseg, grad_rgb, state, lr_sigma=0.1, lr_sh=0.01, alpha=0.99, eps=1e-8,
                         bg=(1.0, 1.0, 1.0), t_stop=1e-4, leaf_count=None, records=None):
        """Adjoint and RMSProp step in one call (no dense gradient arrays)."""
        op = _opts(bg, t_stop)
        p = L.dot_rmsprop_params(lr_sigma=lr_sigma, lr_sh=lr_sh, alpha=alpha, eps=eps)
        L.check(self.lib.dot_render_backward_rmsprop(self.handle, C.byref(rays.struct), C.byref(op), _ptr(rgb),
                                                     _ptr(nseg), _ptr(grad_rgb), _ptr(state["v_sigma"]),
                                                     _ptr(state["v_sh"]), C.byref(p), _ptr(leaf_count), _ptr(records),
                                                     C.c_size_t(records.numel() if records is not None else 0),
                                                     _stream()))

    def backward_adam(self, rays, rgb, nseg, grad_rgb, state, step, lr_sigma=0.1, lr_sh=0.01, beta1=0.9,
                      beta2=0.999, eps=1e-8, bg=(1.0, 1.0, 1.0), t_stop=1e-4, leaf_count=None, records=None):
        """Adjoint and Adam step (1-based `step`) in one call (no dense gradient arrays)."""
        op = _opts(bg, t_stop)
        p = L.dot_adam_params(lr_sigma=lr_sigma, lr_sh=lr_sh, beta1=beta1, beta2=beta2, eps=eps, step=int(step))
        L.check(self.lib.dot_render_backward_adam(self.handle, C.byref(rays.struct), C.byref(op), _ptr(rgb),
                                                  _ptr(nseg), _ptr(grad_rgb), _ptr(state["m_sigma"]),
                                                  _ptr(state["v_sigma"]), _ptr(state["m_sh"]), _ptr(state["v_sh"]),
                                                  C.byref(p), _ptr(leaf_count), _ptr(records),
                                                  C.c_size_t(records.numel() if records is not None else 0),
                                                  _stream()))

    def rmsprop_state(self):
        Ln = self.n_leaves
        z = lambda *s: torch.zeros(s, dtype=torch.float32, device=self.device)
        return dict(v_sigma=z(Ln), v_sh=z(Ln, 3, self.K))

    def sigma_signal(self, out=None):
        """The density signal max(sigma, 0) per leaf (FP32 [L])."""
        if out is None:
            out = torch.empty(self.n_leaves, dtype=torch.float32, device=self.device)
        L.check(self.lib.dot_sigma_signal(self.handle, _ptr(out), _stream()))
        return out

    def quantize_sh(self, bits=16):
        """Median-cut palette compression of the SH rows (in place; storage becomes 'pal16')."""
        L.check(self.lib.dot_quantize_sh(self.handle, int(bits), _stream()))

    def set_links(self, enable=True):
        """Keep or drop the face-neighbour links of the leaf walk (rendered values do not depend on them)."""
        L.check(self.lib.dot_set_links(self.handle, 1 if enable else 0, _stream()))

    def links_view(self):
        """The face-neighbour links as an int32 view [L, 6] (uint32 bits), or None when the tree has none."""
        i = self.info()
        if not i.links:
            return None
        Ln = int(i.n_leaves)
        return self.alloc.tensor(i.links, Ln * 24).view(torch.int32).view(Ln, 6)

    def palette_views(self):
        """(index [L] int16 view of the uint16 indices, palette [2^bits, 3, K] FP16) of a 'pal16' tree."""
        i = self.info()
        if int(i.storage) != L.DOT_PAL16:
            raise ValueError("not a palette-compressed tree")
        Ln, P, st = int(i.n_leaves), 1 << int(i.palette_bits), int(i.sh_stride)
        idx = self.alloc.tensor(i.sh, Ln * 2).view(torch.int16)
        pal = self.alloc.tensor(i.palette, P * st * 2).view(torch.float16).view(P, st)[:, :3 * self.K]
        return idx, pal.unflatten(1, (3, self.K))

    def export(self):
        i = self.info()
        I, Ln = int(i.n_internal), int(i.n_leaves)
        child = np.empty((I, 8), np.int32)
        sigma = np.empty(Ln, np.float32)
        sh = np.empty((Ln, 3, self.K), np.float32)
        depth = np.empty(Ln, np.uint8)
        L.check(self.lib.dot_export(self.handle, child.ctypes.data if I else None, sigma.ctypes.data,
                                    sh.ctypes.data, depth.ctypes.data, _stream()))
        return dict(child=child, sigma=sigma, sh=sh, depth=depth)


def pixel_batch(ray_ids, width, height, n_cams, workspace=None, out=None):
    """(cam_idx int32, pix_idx int32, ray_ids int64) of the flat pixel ids
    `ray_ids` (int64 device [n]) in screen-tile order; `workspace` (uint8
    device tensor) is reused when large enough, and so are the three outputs
    of a previous call passed as `out` when their size is n.  Returns also the
    workspace."""
    lib = L.load()
    n = int(ray_ids.shape[0])
    assert ray_ids.dtype == torch.int64 and ray_ids.is_contiguous()
    need = _pixel_batch_workspace(n, int(width), int(height), int(n_cams))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=ray_ids.device)
    if out is not None and out[0].shape[0] == n:
        cam, pix, ids = out
    else:
        cam = torch.empty(n, dtype=torch.int32, device=ray_ids.device)
        pix = torch.empty(n, dtype=torch.int32, device=ray_ids.device)
        ids = torch.empty(n, dtype=torch.int64, device=ray_ids.device)
    L.check(lib.dot_pixel_batch(_ptr(ray_ids), C.c_int64(n), int(width), int(height), int(n_cams), _ptr(cam),
                                _ptr(pix), _ptr(ids), _ptr(workspace), C.c_size_t(workspace.numel()), _stream()))
    return cam, pix, ids, workspace


@functools.lru_cache(maxsize=64)
def _pixel_batch_workspace(n, width, height, n_cams):
    return int(L.load().dot_pixel_batch_workspace(n, width, height, n_cams))


def mse_loss(pred, target, target_idx=None, grad=True, loss=True, grad_out=None):
    """(loss, grad_rgb) of pred [n,3] against target rows (target_idx: int64 [n]
    or None); either may be skipped.  loss is a device float64 scalar."""
    n = pred.shape[0]
    if grad and grad_out is not None and grad_out.shape == pred.shape:
        g = grad_out
    else:
        g = torch.empty_like(pred) if grad else None
    lo = torch.empty((), dtype=torch.float64, device=pred.device) if loss else None
    if target_idx is not None:
        assert target_idx.dtype == torch.int64 and target_idx.shape[0] == n
    L.check(L.load().dot_mse_loss(_ptr(pred), _ptr(target), _ptr(target_idx), C.c_int64(n), _ptr(g), _ptr(lo),
                                  _stream()))
    return lo, g


class FusedAdam:
    """Adam on a tree's sigma and SH planes, applied inside the adjoint's
    per-leaf reduction when passed to render_autograd (the dense gradients
    are never formed); holds the moments and the 1-based step count."""

    def __init__(self, tree, lr_sigma=0.1, lr_sh=0.01, beta1=0.9, beta2=0.999, eps=1e-8):
        self.tree = tree
        self.state = tree.adam_state()
        self.step = 0
        self.hp = dict(lr_sigma=lr_sigma, lr_sh=lr_sh, beta1=beta1, beta2=beta2, eps=eps)

    def backward_step(self, rays, rgb, nseg, grad_rgb, bg, t_stop, leaf_count, records):
        self.step += 1
        self.tree.backward_adam(rays, rgb, nseg, grad_rgb, self.state, self.step, bg=bg, t_stop=t_stop,
                                leaf_count=leaf_count, records=records, **self.hp)


class FusedRMSProp:
    """RMSProp (Sec. 3.3) applied inside the adjoint's per-leaf reduction; see FusedAdam."""

    def __init__(self, tree, lr_sigma=0.1, lr_sh=0.01, alpha=0.99, eps=1e-8):
        self.tree = tree
        self.state = tree.rmsprop_state()
        self.hp = dict(lr_sigma=lr_sigma, lr_sh=lr_sh, alpha=alpha, eps=eps)

    def backward_step(self, rays, rgb, nseg, grad_rgb, bg, t_stop, leaf_count, records):
        self.tree.backward_rmsprop(rays, rgb, nseg, grad_rgb, self.state, bg=bg, t_stop=t_stop,
                                   leaf_count=leaf_count, records=records, **self.hp)


class DotRender(torch.autograd.Function):
    """C = render(sigma, sh; rays) with the hand-written adjoint as backward.

    ``sigma``/``sh`` are the tree's plane views (see Octree.plane_views); the
    gradients returned are dense FP32 [L] and [L,3,K].  A ``signal`` buffer, if
    given, receives the fused training signal of the forward pass.  On an FP32
    tree the forward is the training forward: it also counts each leaf's
    segments and records up to ``record_segments`` segments per ray, which the
    adjoint replays instead of traversing the tree again (rays with more are
    re-traversed for the rest); ``record_segments=0`` or reduced-precision
    leaves give the plain forward and an adjoint by re-traversal.  The records
    live in a buffer the tree keeps between calls, unless an earlier forward's
    records still wait for their backward.  With ``optimizer`` (FusedAdam or FusedRMSProp) the
    backward applies that optimiser step to the planes inside the adjoint and
    returns no gradient for them."""

    @staticmethod
    def forward(ctx, sigma, sh, tree, rays, bg, t_stop, signal=None, signal_mode="max", record_segments=96,
                optimizer=None):
        cnt = rec = None
        if tree.storage == "f32" and record_segments > 0:
            rec = tree._take_records(rays.n_rays, record_segments)
            rgb, nseg, cnt = tree.render_train(rays, bg=bg, t_stop=t_stop, signal=signal, signal_mode=signal_mode,
                                               records=rec)
        else:
            rgb, nseg = tree.render(rays, bg=bg, t_stop=t_stop, nseg=True, signal=signal, signal_mode=signal_mode)
        ctx.save_for_backward(rgb, nseg)
        ctx.tree, ctx.rays, ctx.bg, ctx.t_stop = tree, rays, bg, t_stop
        ctx.cnt, ctx.rec, ctx.optimizer = cnt, rec, optimizer
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        rgb, nseg = ctx.saved_tensors
        tree = ctx.tree
        g = grad_rgb.contiguous().float()
        if ctx.optimizer is not None:
            ctx.optimizer.backward_step(ctx.rays, rgb, nseg, g, ctx.bg, ctx.t_stop, ctx.cnt, ctx.rec)
            gs = gh = None
        else:
            Ln = tree.n_leaves
            gs = torch.zeros(Ln, dtype=torch.float32, device=rgb.device)
            gh = torch.zeros((Ln, 3, tree.K), dtype=torch.float32, device=rgb.device)
            tree.backward(ctx.rays, rgb, nseg, g, gs, gh, bg=ctx.bg, t_stop=ctx.t_stop, leaf_count=ctx.cnt,
                          records=ctx.rec)
        tree._release_records(ctx.rec)
        ctx.cnt = ctx.rec = ctx.optimizer = None
        return gs, gh, None, None, None, None, None, None, None, None


class MSELoss(torch.autograd.Function):
    """Mean squared error of pred [n, 3] against target rows (Alg. 1's loss);
    the loss is a float64 device scalar (dot_mse_loss).  The backward is one
    kernel (dot_mse_grad) that scales the gradient by the upstream gradient
    where it lies on the device, so no host value is read."""

    @staticmethod
    def forward(ctx, pred, target, target_idx=None):
        loss, _ = mse_loss(pred, target, target_idx, grad=False)
        ctx.save_for_backward(pred, target, target_idx)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        pred, target, target_idx = ctx.saved_tensors
        scale = grad_loss if grad_loss.dtype == torch.float64 else grad_loss.to(torch.float64)   # one element
        g = torch.empty_like(pred)
        L.check(L.load().dot_mse_grad(_ptr(pred), _ptr(target), _ptr(target_idx), C.c_int64(pred.shape[0]),
                                      _ptr(scale), _ptr(g), _stream()))
        return g, None, None


def mse_loss_autograd(pred, target, target_idx=None):
    return MSELoss.apply(pred, target, target_idx)


def render_autograd(tree, sigma, sh, rays, bg=(1.0, 1.0, 1.0), t_stop=1e-4, signal=None, signal_mode="max",
                    record_segments=96, optimizer=None):
    return DotRender.apply(sigma, sh, tree, rays, bg, t_stop, signal, signal_mode, record_segments, optimizer)
