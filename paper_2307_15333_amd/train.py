"""The refinement-training loop of DOT (Alg. 1) over a device-resident octree.

One epoch permutes the training rays, then for every batch of the permuted
order renders the batch (fusing the training signal Q into the forward pass
when this epoch ends with a refinement), takes the MSE against the ground-truth
pixels, runs the hand-written adjoint and one optimiser step (RMSProp as in
Sec. 3.3, or Adam).  Every `interval` epochs (the structure is frozen for T
epochs in between, Sec. 3.3) the octree is refined from the epoch's signal:
recursive or one-level pruning of groups whose signal is at most tau, then
subdivision of the top gamma fraction of leaves (Sec. 3.2), with fused
features or, for the ablation without fusion, fresh zero-valued leaves.  The
optimiser state restarts from zero after a refinement, since the leaf set
changed.

Everything per ray and per leaf runs in libdot's kernels (a batch is put in
screen-tile order by dot_pixel_batch before it is rendered, so a wave traces
neighbouring pixels); this module only sequences the calls and slices the
permuted ray order into batches.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import core


@dataclasses.dataclass
class TrainConfig:
    epochs: int = 100
    interval: int = 20              # T: epochs between refinements (Sec. 4.1)
    batch_rays: int = 1 << 18
    optimizer: str = "rmsprop"      # "rmsprop" (Sec. 3.3) or "adam"
    lr_sigma: float = 0.1           # Sec. 4.1
    lr_sh: float = 0.01
    alpha: float = 0.99             # RMSProp square-average decay
    beta1: float = 0.9              # Adam
    beta2: float = 0.999
    eps: float = 1e-8
    signal: str = "max"             # "max" / "sum" of ray weights (Q), or "sigma" (the Pr_sigma ablation)
    tau: float = 1e-3               # prune groups whose signal is <= tau (Sec. 3.2)
    gamma: float = 0.01             # subdivide the top gamma fraction of leaves
    prune_le: bool = True
    max_depth: int = 10
    recursive: bool = False
    reinit: bool = False            # ablation: new leaves start at zero instead of fused values
    refine: bool = True
    fused: bool = True              # the optimiser step applied inside the adjoint's per-leaf reduction
    # upper bound on the segments per ray the forward records for the adjoint's replay; each epoch's first batch
    # sets the capacity to 5/4 of its longest ray (a ray with more is re-traversed for the rest by a few
    # long-running waves at the end of the adjoint); the buffer holds n x capacity x 28 B of device memory
    record_segments: int = 256
    bg: tuple = (1.0, 1.0, 1.0)
    t_stop: float = 1e-4
    seed: int = 0


class Trainer:
    """Alg. 1 on `tree` (FP32 storage) against multi-view targets.

    cams: camera records (all of one size W x H); targets: float32 [n_cams, H, W, 3]
    (host or device)."""

    def __init__(self, tree, cams, targets, cfg: TrainConfig):
        if tree.storage != "f32":
            raise ValueError("training needs FP32 leaf storage")
        if cfg.signal not in ("max", "sum", "sigma"):
            raise ValueError(f"unknown signal {cfg.signal!r}")
        if cfg.optimizer not in ("rmsprop", "adam"):
            raise ValueError(f"unknown optimizer {cfg.optimizer!r}")
        self.tree = tree
        self.cfg = cfg
        self.device = tree.device
        cams = np.asarray(cams)
        self.n_cams = len(cams)
        self.W, self.H = int(cams[0]["width"]), int(cams[0]["height"])
        _, self.cams_raw = core.Rays._cams_tensor(cams, self.device)
        self.targets = torch.as_tensor(targets, dtype=torch.float32).to(self.device).reshape(-1, 3).contiguous()
        self.n_rays = self.n_cams * self.W * self.H
        if self.targets.shape[0] != self.n_rays:
            raise ValueError("targets must hold one RGB value per pixel of every camera")
        self.gen = torch.Generator(device=self.device)
        self.gen.manual_seed(int(cfg.seed))
        self.epoch = 0
        self.opt_step = 0
        self._ws = None
        self._pb = self._fw = self._grad = None     # per-batch buffers, reused while the batch size stays
        self._rec = None        # segment records of the current batch (forward -> adjoint)
        self._rec_cap = None    # records per ray, from the longest ray of an epoch's first batch
        self._size_records = True
        self._reset_optimizer()

    def _reset_optimizer(self):
        t = self.tree
        self.state = t.rmsprop_state() if self.cfg.optimizer == "rmsprop" else t.adam_state()
        self.gs = self.gh = None      # dense gradients, for the unfused optimiser steps only
        self._cnt = None              # per-leaf segment counts of the current batch
        self.opt_step = 0

    def permutation(self):
        return torch.randperm(self.n_rays, generator=self.gen, device=self.device)

    def step(self, idx, signal=None):
        """One optimisation step on the rays idx (int64 device tensor of pixel
        indices into the flattened [n_cams, H, W] images).  Returns the batch
        loss as a device float64 scalar."""
        c = self.cfg
        # the batch's buffers are kept from one step to the next (same batch size)
        cam, pix, ids, self._ws = core.pixel_batch(idx.contiguous(), self.W, self.H, self.n_cams, self._ws,
                                                   out=self._pb)
        self._pb = (cam, pix, ids)
        rays = core.Rays.pixels_device(self.cams_raw, self.n_cams, cam, pix)
        mode = "sum" if c.signal == "sum" else "max"
        # the training forward also counts each leaf's segments and records the
        # composited segments, so the adjoint neither traverses nor refetches
        # room for the longest ray seen at the first batch of the epoch (with a
        # margin), at most record_segments; a longer ray is re-traversed for
        # the rest of its segments
        cap = c.record_segments if self._rec_cap is None else self._rec_cap
        need = core.Octree.records_bytes(idx.shape[0], cap)
        if self._rec is None or self._rec.numel() < need or self._rec.numel() > 2 * need:
            self._rec = torch.empty(need, dtype=torch.uint8, device=self.device)
        rgb, nseg, self._cnt = self.tree.render_train(rays, bg=c.bg, t_stop=c.t_stop, signal=signal, signal_mode=mode,
                                                      leaf_count=self._cnt, records=self._rec[:need], out=self._fw)
        self._fw = (rgb, nseg)
        if self._size_records:
            self._size_records = False
            self._rec_cap = min(c.record_segments, max(8, (int(nseg.max()) * 5 // 4 + 7) // 8 * 8))
        loss, grad = core.mse_loss(rgb, self.targets, ids, grad_out=self._grad)
        self._grad = grad
        self.opt_step += 1
        if c.fused:
            # adjoint and update in one call: the gradient never exists as dense arrays
            if c.optimizer == "rmsprop":
                self.tree.backward_rmsprop(rays, rgb, nseg, grad, self.state, lr_sigma=c.lr_sigma, lr_sh=c.lr_sh,
                                           alpha=c.alpha, eps=c.eps, bg=c.bg, t_stop=c.t_stop, leaf_count=self._cnt,
                                           records=self._rec[:need])
            else:
                self.tree.backward_adam(rays, rgb, nseg, grad, self.state, self.opt_step, lr_sigma=c.lr_sigma,
                                        lr_sh=c.lr_sh, beta1=c.beta1, beta2=c.beta2, eps=c.eps, bg=c.bg,
                                        t_stop=c.t_stop, leaf_count=self._cnt, records=self._rec[:need])
            return loss
        if self.gs is None:
            t = self.tree
            self.gs = torch.zeros(t.n_leaves, dtype=torch.float32, device=self.device)
            self.gh = torch.zeros((t.n_leaves, 3, t.K), dtype=torch.float32, device=self.device)
        else:
            self.gs.zero_()
            self.gh.zero_()
        self.tree.backward(rays, rgb, nseg, grad, self.gs, self.gh, bg=c.bg, t_stop=c.t_stop, leaf_count=self._cnt,
                           records=self._rec[:need])
        if c.optimizer == "rmsprop":
            self.tree.rmsprop_step(self.gs, self.gh, self.state, lr_sigma=c.lr_sigma, lr_sh=c.lr_sh,
                                   alpha=c.alpha, eps=c.eps)
        else:
            self.tree.adam_step(self.gs, self.gh, self.state, self.opt_step, lr_sigma=c.lr_sigma, lr_sh=c.lr_sh,
                                beta1=c.beta1, beta2=c.beta2, eps=c.eps)
        return loss

    def run_epoch(self, perm=None):
        """One epoch of Alg. 1 (1-based epoch number i = self.epoch after the
        call); refines when i is a multiple of the interval.  Returns a dict
        with the batch losses (host) and, after a refinement, its statistics."""
        c = self.cfg
        self.epoch += 1
        refine_now = c.refine and c.interval > 0 and self.epoch % c.interval == 0
        if perm is None:
            perm = self.permutation()
        else:
            perm = torch.as_tensor(perm, dtype=torch.int64).to(self.device)
            if perm.shape[0] != self.n_rays:
                raise ValueError("a permutation must cover every training ray")
        self._size_records = True
        signal = None
        if refine_now and c.signal != "sigma":
            signal = torch.zeros(self.tree.n_leaves, dtype=torch.float32, device=self.device)
        losses = []
        for b in range(0, self.n_rays, c.batch_rays):
            losses.append(self.step(perm[b:b + c.batch_rays], signal))
        out = dict(epoch=self.epoch, losses=torch.stack(losses).cpu().numpy() if losses else np.zeros(0))
        if refine_now:
            if c.signal == "sigma":
                signal = self.tree.sigma_signal()
            out["signal"] = signal
            out["refine"] = self.tree.refine(signal, prune_tau=c.tau, sample_frac=c.gamma, max_depth=c.max_depth,
                                             prune_le=c.prune_le, recursive=c.recursive, reinit=c.reinit)
            self._reset_optimizer()
        out["leaves"] = self.tree.n_leaves
        return out

    def train(self, epochs=None, callback=None):
        hist = []
        for _ in range(self.cfg.epochs if epochs is None else epochs):
            r = self.run_epoch()
            r.pop("signal", None)
            hist.append(r)
            if callback is not None:
                callback(r)
        return hist
