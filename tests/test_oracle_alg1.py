"""Pins of the training-loop oracle (Alg. 1) and its per-step pieces.

The loss and optimiser pieces are checked against PyTorch's own CPU
implementations of the same definitions (MSE, RMSProp, Adam) and against
closed forms; the loop is checked through properties that any correct
implementation of Alg. 1 has: order-independence of the MAX signal, the
fixed point at a perfect fit, a falling loss, and the refinement counts.
None of these calls the HIP library.
"""
import math

import numpy as np
import pytest
import torch

from oracle import alg1 as A
from oracle import oracle as O
from paper_2307_15333_amd import synth


def test_mse_loss_matches_torch_and_its_gradient():
    rng = np.random.default_rng(0)
    pred = rng.normal(size=(37, 3))
    tgt = rng.normal(size=(37, 3))
    loss, grad = A.mse_loss(pred, tgt)
    p = torch.tensor(pred, dtype=torch.float64, requires_grad=True)
    ref = torch.nn.functional.mse_loss(p, torch.tensor(tgt, dtype=torch.float64))
    ref.backward()
    assert loss == pytest.approx(ref.item(), rel=1e-14)
    np.testing.assert_allclose(grad, p.grad.numpy(), rtol=1e-13, atol=0)
    assert A.mse_loss(pred, pred)[0] == 0.0


def test_rmsprop_matches_torch_rmsprop():
    rng = np.random.default_rng(1)
    theta0 = rng.normal(size=50)
    grads = [rng.normal(size=50) * 10.0 ** rng.uniform(-6, 1, size=50) for _ in range(6)]
    for lr, alpha, eps in ((0.1, 0.99, 1e-8), (0.01, 0.9, 1e-3)):
        p = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64))
        opt = torch.optim.RMSprop([p], lr=lr, alpha=alpha, eps=eps)
        th, v = theta0.copy(), np.zeros(50)
        for g in grads:
            p.grad = torch.tensor(g, dtype=torch.float64)
            opt.step()
            th, v = A.rmsprop(th, g, v, lr, alpha, eps)
        np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_rmsprop_constant_gradient_closed_form():
    # With a constant gradient g from v = 0, v_t = (1 - alpha^t) g^2, so step t
    # moves theta by lr g / (|g| sqrt(1 - alpha^t) + eps).
    g, lr, alpha, eps = np.array([0.3, -2.0, 1e-5]), 0.1, 0.9, 1e-8
    th, v = np.zeros(3), np.zeros(3)
    expect = np.zeros(3)
    for t in range(1, 8):
        th, v = A.rmsprop(th, g, v, lr, alpha, eps)
        expect -= lr * g / (np.abs(g) * math.sqrt(1 - alpha ** t) + eps)
        np.testing.assert_allclose(v, (1 - alpha ** t) * g * g, rtol=1e-13)
    np.testing.assert_allclose(th, expect, rtol=1e-12)


def test_adam_matches_torch_adam():
    rng = np.random.default_rng(4)
    theta0 = rng.normal(size=50)
    grads = [rng.normal(size=50) * 10.0 ** rng.uniform(-6, 1, size=50) for _ in range(7)]
    for lr, b1, b2, eps in ((0.1, 0.9, 0.999, 1e-8), (0.01, 0.8, 0.99, 1e-4)):
        p = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64))
        opt = torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps)
        th, m, v = theta0.copy(), np.zeros(50), np.zeros(50)
        for t, g in enumerate(grads, start=1):
            p.grad = torch.tensor(g, dtype=torch.float64)
            opt.step()
            th, m, v = A.adam(th, g, m, v, t, lr, b1, b2, eps)
            np.testing.assert_allclose(m, opt.state[p]["exp_avg"].numpy(), rtol=1e-13, atol=0)
            np.testing.assert_allclose(v, opt.state[p]["exp_avg_sq"].numpy(), rtol=1e-13, atol=0)
        np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)
    with pytest.raises(ValueError):
        A.adam(theta0, grads[0], np.zeros(50), np.zeros(50), 0, 0.1, 0.9, 0.999, 1e-8)


def test_adam_constant_gradient_closed_form():
    # With a constant gradient g from m = v = 0: m_t = (1 - b1^t) g and
    # v_t = (1 - b2^t) g^2, so the bias-corrected moments are g and g^2 and
    # every step moves theta by exactly lr g / (|g| + eps).  A bias correction
    # off by one step, or the two betas swapped, breaks this.
    g, lr, b1, b2, eps = np.array([0.3, -2.0, 1e-5]), 0.1, 0.9, 0.999, 1e-8
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    expect = np.zeros(3)
    for t in range(1, 9):
        th, m, v = A.adam(th, g, m, v, t, lr, b1, b2, eps)
        expect -= lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(m, (1 - b1 ** t) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12)
        np.testing.assert_allclose(th, expect, rtol=1e-12)
    # a zero gradient after a constant one: the first moment decays, theta keeps moving
    th2, m2, v2 = A.adam(th, np.zeros(3), m, v, 9, lr, b1, b2, eps)
    want = th - lr * (b1 * m / (1 - b1 ** 9)) / (np.sqrt(b2 * v / (1 - b2 ** 9)) + eps)
    np.testing.assert_allclose(th2, want, rtol=1e-13)
    assert np.all(th2 != th)


def test_sigma_signal_is_the_clamped_density():
    s = np.array([-3.0, -0.0, 0.0, 1e-30, 2.5])
    np.testing.assert_array_equal(A.sigma_signal(s), [0.0, 0.0, 0.0, 1e-30, 2.5])


def _setup(n_views=3, size=16, seed=5):
    sc = synth.sphere_scene()
    cams = synth.random_sphere_cameras(n_views, 4.0, size, size, seed=seed)
    o, d = O.camera_rays(cams)
    return sc, cams, o.reshape(-1, 3), d.reshape(-1, 3)


def _args(sc):
    return (sc.child, sc.sigma64, sc.sh32, sc.degree, sc.bbox_min, sc.bbox_size)


def test_loop_adam_steps_are_the_adam_pieces_and_restart_after_refinement():
    # The loop's Adam is the per-step Adam with a step count that starts at 1
    # and starts again, with zero moments, after a refinement.  Two epochs of
    # two batches, a refinement after each that changes no leaf (tau below
    # every signal, gamma = 0) but rounds the values to the FP32 storage; the
    # density's learning rate is 0, so the rays' segments stay fixed and the SH
    # updates can be replayed by hand from the pieces.
    sc, cams, o, d = _setup(n_views=1, size=8)
    n = o.shape[0]
    tgt = np.random.default_rng(9).uniform(size=(n, 3))
    perm = [np.arange(n), np.arange(n)]
    st, hist = A.train(*_args(sc), o, d, tgt, perm, n // 2, interval=1, lr_sigma=0.0, lr_sh=0.05, tau=-1.0,
                       gamma=0.0, optimizer="adam", eps=1e-6)
    assert all(h["merged"] == 0 and h["subdivided"] == 0 for h in hist)
    sh = sc.sh32.astype(np.float64)
    for epoch in range(2):
        m, v = np.zeros_like(sh), np.zeros_like(sh)
        for t, b in enumerate((slice(0, n // 2), slice(n // 2, n)), start=1):
            T = O.OracleTree(sc.child, sc.sigma64, sh, sc.degree, sc.bbox_min, sc.bbox_size)
            r = O.render(T, o[b], d[b])
            _, g = A.mse_loss(r["rgb"], tgt[b])
            _, gh = O.backward(T, o[b], d[b], g)
            sh, m, v = A.adam(sh, gh, m, v, t, 0.05, 0.9, 0.999, 1e-6)
        sh = sh.astype(np.float32).astype(np.float64)      # the refinement's storage rounding
    # equal up to the gradient's summation order (the oracle's threads) and an
    # FP32 rounding that order can flip; a step count or moments carried over
    # the refinement would move the SH by ~1e-2
    np.testing.assert_allclose(st["sh"], sh, rtol=1e-6, atol=1e-7)
    assert np.abs(st["sh"] - sc.sh32).max() > 1e-2
    np.testing.assert_array_equal(st["sigma"], sc.sigma64.astype(np.float32))
    with pytest.raises(ValueError):
        A.train(*_args(sc), o, d, tgt, perm, n, optimizer="sgd")


def test_loop_signal_and_losses_do_not_depend_on_the_ray_order():
    # lr = 0 freezes the leaves, so the epoch's MAX signal is the max over all
    # rays of one full render whatever the permutation and batch size, and
    # each batch loss is the MSE of the full render's rows.
    sc, cams, o, d = _setup()
    n = o.shape[0]
    tgt = np.random.default_rng(2).uniform(size=(n, 3))
    full = O.render(O.OracleTree.from_scene(sc), o, d, signal=True)
    for perm_seed, batch in ((0, 100), (1, n)):
        perm = synth.ray_permutations(n, 1, perm_seed)
        _, hist = A.train(*_args(sc), o, d, tgt, perm, batch, interval=1, lr_sigma=0.0, lr_sh=0.0,
                          tau=-1.0, gamma=0.0)
        h = hist[0]
        np.testing.assert_array_equal(h["sig"], full["sig"])
        np.testing.assert_array_equal(h["sig_lo"], full["sig_lo"])
        exp = [A.mse_loss(full["rgb"][perm[0][b:b + batch]], tgt[perm[0][b:b + batch]])[0]
               for b in range(0, n, batch)]
        np.testing.assert_allclose(h["losses"], exp, rtol=1e-13)
        assert h["merged"] == 0 and h["subdivided"] == 0


def test_loop_sum_signal_is_the_sum_over_batches():
    sc, cams, o, d = _setup()
    n = o.shape[0]
    tgt = np.zeros((n, 3))
    full = O.render(O.OracleTree.from_scene(sc), o, d, signal=True, signal_mode="sum")
    _, hist = A.train(*_args(sc), o, d, tgt, synth.ray_permutations(n, 1, 3), 97, interval=1, lr_sigma=0.0,
                      lr_sh=0.0, tau=-1.0, gamma=0.0, signal="sum")
    np.testing.assert_allclose(hist[0]["sig"], full["sig"], rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("optimizer", ["rmsprop", "adam"])
def test_loop_perfect_fit_is_a_fixed_point(optimizer):
    # Targets rendered from the starting tree: every residual, hence every
    # gradient and update, is exactly zero.  A wrong target row fails this.
    sc, cams, o, d = _setup()
    n = o.shape[0]
    tgt = O.render(O.OracleTree.from_scene(sc), o, d)["rgb"]
    st, hist = A.train(*_args(sc), o, d, tgt, synth.ray_permutations(n, 2, 4), 128, interval=0,
                       optimizer=optimizer)
    assert all(np.all(h["losses"] == 0.0) for h in hist)
    np.testing.assert_array_equal(st["sigma"], sc.sigma64)
    np.testing.assert_array_equal(st["sh"], sc.sh32.astype(np.float64))


@pytest.mark.parametrize("optimizer", ["rmsprop", "adam"])
def test_loop_reduces_the_loss(optimizer):
    sc, cams, o, d = _setup(n_views=4)
    n = o.shape[0]
    tgt = O.render(O.OracleTree.from_scene(sc), o, d)["rgb"]
    start = synth.perturb_sh(sc, std=0.3, seed=7)
    _, hist = A.train(*_args(start), o, d, tgt, synth.ray_permutations(n, 6, 5), 256, interval=0,
                      lr_sigma=0.01, lr_sh=0.01, optimizer=optimizer)
    first, last = hist[0]["losses"].mean(), hist[-1]["losses"].mean()
    assert last < 0.5 * first


@pytest.mark.parametrize("recursive,reinit,signal", [(False, False, "max"), (True, True, "sigma")])
def test_loop_refinement_counts(recursive, reinit, signal):
    sc, cams, o, d = _setup()
    n = o.shape[0]
    tgt = O.render(O.OracleTree.from_scene(sc), o, d)["rgb"]
    start = synth.perturb_sh(sc, std=0.2, seed=8)
    L0 = sc.sigma64.shape[0]
    st, hist = A.train(*_args(start), o, d, tgt, synth.ray_permutations(n, 2, 6), 256, interval=2, tau=1e-3,
                       gamma=0.02, recursive=recursive, reinit=reinit, signal=signal, max_depth=6)
    h = hist[1]
    assert h["k"] == math.floor(0.02 * L0)
    assert h["merged"] > 0 and h["subdivided"] > 0
    # each merged group removes 7 leaves net (8 -> 1) at one level, each split adds 7
    L1 = st["sigma"].shape[0]
    assert h["leaves"] == L1
    if not recursive:
        assert L1 == L0 - 7 * h["merged"] + 7 * h["subdivided"]
    assert st["child"].shape[0] * 8 + 1 == st["child"].shape[0] + L1  # full octree: I*8 + 1 = I + L
