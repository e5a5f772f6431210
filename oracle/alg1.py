"""FP64 oracle of the DOT training loop (Alg. 1) and its per-step pieces.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; the product path never
imports it.  Each piece is the plain definition, in the order Alg. 1 takes the
steps:

  * ``mse_loss``      -- the photometric loss of a ray batch (Alg. 1, the MSE
                         of the prediction against the ground truth), mean over
                         rays and colour channels, and its gradient.
  * ``rmsprop``       -- the optimiser of Sec. 3.3 (RMSProp): a decayed mean of
                         squared gradients scales each parameter's step.
  * ``adam``          -- Adam (Kingma & Ba, 2015), the optimiser the
                         differentiable training-step workload uses on the same
                         parameters: decayed first and second moments, each
                         divided by its bias correction 1 - beta^t.
  * ``sigma_signal``  -- the density used as the refinement signal in the
                         Pr_sigma ablation (Sec. 3.1, Tab. 3): max(sigma, 0).
  * ``train``         -- epochs of Alg. 1: for each batch of the given ray
                         permutation render (with the signal Q), MSE, adjoint,
                         optimiser step (RMSProp, or Adam); every T-th epoch prune(Q, tau) and
                         sample(Q, gamma) through the refinement oracle.

Parameters are kept in FP64 between steps; the refinement oracle rounds the
refined leaves to the FP32 storage of a trainable tree.  Random draws (the ray
permutations) are inputs.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def mse_loss(pred, target):
    """loss = mean over all n*3 entries of (pred - target)^2; grad = 2 (pred - target) / (3n)."""
    e = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    m = e.size
    if m == 0:
        return 0.0, e
    return float(np.sum(e * e) / m), 2.0 * e / m


def rmsprop(theta, g, v, lr, alpha, eps):
    """v <- alpha v + (1 - alpha) g^2; theta <- theta - lr g / (sqrt(v) + eps)."""
    v = alpha * v + (1.0 - alpha) * g * g
    return theta - lr * g / (np.sqrt(v) + eps), v


def adam(theta, g, m, v, t, lr, beta1, beta2, eps):
    """Step t >= 1: m <- beta1 m + (1 - beta1) g; v <- beta2 v + (1 - beta2) g^2;
    theta <- theta - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
    Returns (theta, m, v)."""
    if t < 1:
        raise ValueError("Adam steps are numbered from 1")
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def sigma_signal(sigma):
    return np.maximum(np.asarray(sigma, np.float64), 0.0)


def train(child, sigma, sh, degree, bbox_min, bbox_size, origins, dirs, targets, perms, batch, interval=20,
          tau=1e-3, gamma=0.01, prune_le=True, max_depth=10, recursive=False, reinit=False, signal="max",
          lr_sigma=0.1, lr_sh=0.01, alpha=0.99, eps=1e-8, bg=(1.0, 1.0, 1.0), t_stop=1e-4, optimizer="rmsprop",
          betas=(0.9, 0.999)):
    """Run len(perms) epochs (epoch i = 1, 2, ...; refine when i % interval == 0).

    origins/dirs/targets: [n, 3] per training ray; perms: list of index arrays
    (each a permutation of range(n)).  Returns (state, history): state holds
    child, sigma, sh (FP64) and depth of the final tree; history one dict per
    epoch with the batch losses, and at a refinement the signal that drove it
    (sig, and bounds sig_lo / sig_hi from the oracle's stopping-rule variants)
    and the refinement counts.  optimizer: "rmsprop" (alpha, eps) or "adam"
    (betas, eps); the optimiser state, and Adam's step count, start again from
    zero after each refinement."""
    if optimizer not in ("rmsprop", "adam"):
        raise ValueError(optimizer)
    child = np.ascontiguousarray(child, np.int32).reshape(-1, 8)
    sigma = np.array(sigma, np.float64)
    K = (degree + 1) ** 2
    sh = np.array(sh, np.float64).reshape(-1, 3, K)
    origins = np.asarray(origins, np.float64)
    dirs = np.asarray(dirs, np.float64)
    targets = np.asarray(targets, np.float64)
    v_s, v_h = np.zeros_like(sigma), np.zeros_like(sh)
    m_s, m_h = np.zeros_like(sigma), np.zeros_like(sh)
    t_opt = 0
    depth = None
    mode = "sum" if signal == "sum" else "max"
    hist = []
    for i, perm in enumerate(perms, start=1):
        perm = np.asarray(perm, np.int64)
        refine_now = interval > 0 and i % interval == 0
        want_q = refine_now and signal != "sigma"
        q = [np.zeros(sigma.shape[0]) for _ in range(3)] if want_q else None
        losses = []
        for b in range(0, perm.shape[0], batch):
            idx = perm[b:b + batch]
            tree = O.OracleTree(child, sigma, sh, degree, bbox_min, bbox_size)
            r = O.render(tree, origins[idx], dirs[idx], bg=bg, t_stop=t_stop, signal=want_q, signal_mode=mode)
            loss, grad = mse_loss(r["rgb"], targets[idx])
            gs, gh = O.backward(tree, origins[idx], dirs[idx], grad, bg=bg, t_stop=t_stop)
            if optimizer == "rmsprop":
                sigma, v_s = rmsprop(sigma, gs, v_s, lr_sigma, alpha, eps)
                sh, v_h = rmsprop(sh, gh, v_h, lr_sh, alpha, eps)
            else:
                t_opt += 1
                sigma, m_s, v_s = adam(sigma, gs, m_s, v_s, t_opt, lr_sigma, betas[0], betas[1], eps)
                sh, m_h, v_h = adam(sh, gh, m_h, v_h, t_opt, lr_sh, betas[0], betas[1], eps)
            losses.append(loss)
            if want_q:
                for a, key in enumerate(("sig", "sig_lo", "sig_hi")):
                    q[a] = np.maximum(q[a], r[key]) if mode == "max" else q[a] + r[key]
        rec = dict(epoch=i, losses=np.array(losses))
        if refine_now:
            if signal == "sigma":
                s = sigma_signal(sigma)
                rec.update(sig=s, sig_lo=s, sig_hi=s)
            else:
                rec.update(sig=q[0], sig_lo=q[1], sig_hi=q[2])
            tree = O.OracleTree(child, sigma, sh, degree, bbox_min, bbox_size)
            out = O.refine(tree, rec["sig"].astype(np.float32), tau=tau, sample_frac=gamma, max_depth=max_depth,
                           prune_le=prune_le, recursive=recursive, storage="f32", reinit=reinit)
            child = out["child"]
            sigma = out["sigma"].astype(np.float64)
            sh = out["sh"].astype(np.float64)
            depth = out["depth"]
            v_s, v_h = np.zeros_like(sigma), np.zeros_like(sh)
            m_s, m_h = np.zeros_like(sigma), np.zeros_like(sh)
            t_opt = 0
            rec.update(merged=out["merged"], subdivided=out["subdivided"], k=out["k"], depth=depth)
        rec["leaves"] = sigma.shape[0]
        hist.append(rec)
    return dict(child=child, sigma=sigma, sh=sh, depth=depth), hist
