"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/dot.h declares, and rejects malformed input before any
device work with a specific message."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2307_15333_amd import _lib as L
from paper_2307_15333_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "dot.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dot_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(L.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.check_output(["nm", "-D", "--defined-only", L.LIB_PATH]).decode()
    exported = set(re.findall(r" T (dot_[a-z_]+)$", out, flags=re.M))
    assert set(_declared()) <= exported


def test_library_leaves_none_of_its_own_symbols_undefined():
    """Every symbol the library needs from outside is a versioned one of the C/C++ or HIP runtime (or weak): a
    launcher declared with the wrong linkage would show up here unversioned, and fail only when first called."""
    out = subprocess.check_output(["nm", "-D", "--undefined-only", L.LIB_PATH]).decode()
    own = [ln.split()[-1] for ln in out.splitlines()
           if ln.split() and ln.split()[0] == "U" and "@" not in ln.split()[-1]]
    assert own == [], own


def _build(child, sigma, sh, degree=0, n_internal=None, n_leaves=None, storage=L.DOT_F32, bbox=2.0):
    lib = L.load()
    child = np.ascontiguousarray(child, np.int32)
    sigma = np.ascontiguousarray(sigma, np.float32)
    sh = np.ascontiguousarray(sh, np.float32)
    d = L.dot_tree_desc(n_internal=child.shape[0] if n_internal is None else n_internal,
                        n_leaves=sigma.shape[0] if n_leaves is None else n_leaves, sh_degree=degree,
                        child=child.ctypes.data if child.size else None, sigma=sigma.ctypes.data,
                        sh=sh.ctypes.data, bbox_size=bbox)
    h = C.c_void_p()
    rc = lib.dot_build(C.byref(d), storage, None, None, C.byref(h))
    return rc, lib.dot_last_error().decode()


def _tree():
    s = synth.random_tree_scene(3, 0, seed=1)
    return s.child.copy(), s.sigma.copy(), s.sh.copy()


@pytest.mark.parametrize("mutate, msg", [
    (lambda c: c.__setitem__((0, 3), 10 ** 6), "out of range"),
    (lambda c: c.__setitem__((0, 3), c[0, 2]), "referenced twice"),
    (lambda c: c.__setitem__((0, 0), -10 ** 6), "out of range"),
])
def test_build_rejects_malformed_child_arrays(mutate, msg):
    child, sigma, sh = _tree()
    mutate(child)
    rc, err = _build(child, sigma, sh)
    assert rc == L.DOT_EINVAL and msg in err, err


def test_build_rejects_cycles_and_unreachable_nodes():
    child, sigma, sh = _tree()
    # an internal child pointing back at the root is a cycle
    j = int(np.argwhere(child[1:] >= 0)[0][0]) + 1 if (child[1:] >= 0).any() else None
    c2 = child.copy()
    c2[1, 0] = 0
    rc, err = _build(c2, sigma, sh)
    assert rc == L.DOT_EINVAL
    # declaring more leaves than the tree references
    rc, err = _build(child, np.concatenate([sigma, [1.0]]), np.concatenate([sh, sh[:1]]))
    assert rc == L.DOT_EINVAL and "unreachable" in err


def test_build_rejects_leaves_out_of_dfs_order():
    child, sigma, sh = _tree()
    c2 = child.copy()
    leaves = np.argwhere(c2 < 0)
    a, b = leaves[0], leaves[1]
    c2[tuple(a)], c2[tuple(b)] = c2[tuple(b)], c2[tuple(a)]
    rc, err = _build(c2, sigma, sh)
    assert rc == L.DOT_EINVAL and "depth-first" in err


def test_build_rejects_depth_beyond_lattice():
    # a chain of 17 internal nodes
    n = 17
    child = np.empty((n, 8), np.int32)
    leaf = 0
    for i in range(n):
        for o in range(8):
            if o == 0 and i + 1 < n:
                child[i, o] = i + 1
            else:
                child[i, o] = -1 - leaf
                leaf += 1
    # leaves must be numbered in DFS order: renumber by a walk
    order = []

    def walk(i):
        for o in range(8):
            e = child[i, o]
            if e >= 0:
                walk(e)
            else:
                order.append(-1 - e)

    walk(0)
    remap = {old: new for new, old in enumerate(order)}
    child = np.where(child < 0, -1 - np.vectorize(lambda e: remap[-1 - e])(np.minimum(child, -1)), child)
    rc, err = _build(child, np.ones(leaf), np.zeros((leaf, 3, 1)))
    assert rc == L.DOT_EINVAL and "DOT_MAX_DEPTH" in err


def test_build_rejects_bad_arguments():
    child, sigma, sh = _tree()
    rc, err = _build(child, sigma, sh, degree=4)
    assert rc == L.DOT_EINVAL and "sh_degree" in err
    rc, err = _build(child, sigma, sh, storage=7)
    assert rc == L.DOT_EINVAL and "storage" in err
    rc, err = _build(child, sigma, sh, bbox=-1.0)
    assert rc == L.DOT_EINVAL and "bbox_size" in err
    rc, err = _build(np.zeros((0, 8)), np.ones(2), np.zeros((2, 3, 1)))
    assert rc == L.DOT_EINVAL and "exactly one leaf" in err
    lib = L.load()
    h = C.c_void_p()
    assert lib.dot_build(None, 0, None, None, C.byref(h)) == L.DOT_EINVAL
    assert b"desc is NULL" in lib.dot_last_error()


def test_calls_on_null_handles_fail_cleanly():
    lib = L.load()
    assert lib.dot_free(None) == L.DOT_OK
    r = L.dot_rays()
    assert lib.dot_render(None, C.byref(r), None, None, None, None, None) == L.DOT_EINVAL
    assert b"tree is NULL" in lib.dot_last_error()
    info = L.dot_tree_info_t()
    assert lib.dot_tree_info(None, C.byref(info)) == L.DOT_EINVAL
    p = L.dot_refine_params()
    assert lib.dot_refine(None, None, C.byref(p), None, None) == L.DOT_EINVAL
    rp = L.dot_rmsprop_params(lr_sigma=0.1, lr_sh=0.01, alpha=0.99, eps=1e-8)
    assert lib.dot_rmsprop_step(None, None, None, None, None, C.byref(rp), None) == L.DOT_EINVAL
    assert lib.dot_render_backward_rmsprop(None, C.byref(r), None, None, None, None, None, None, C.byref(rp), None,
                                           None, 0, None) == L.DOT_EINVAL
    ap = L.dot_adam_params(lr_sigma=0.1, lr_sh=0.01, beta1=0.9, beta2=0.999, eps=1e-8, step=1)
    assert lib.dot_adam_step(None, None, None, None, None, None, None, C.byref(ap), None) == L.DOT_EINVAL
    assert lib.dot_render_backward_adam(None, C.byref(r), None, None, None, None, None, None, None, None,
                                        C.byref(ap), None, None, 0, None) == L.DOT_EINVAL
    assert b"NULL tree" in lib.dot_last_error()
    assert lib.dot_sigma_signal(None, None, None) == L.DOT_EINVAL


def test_batch_and_loss_argument_checks_need_no_device():
    lib = L.load()
    assert lib.dot_mse_loss(None, None, None, -1, None, None, None) == L.DOT_EINVAL
    assert lib.dot_mse_loss(None, None, None, 5, None, None, None) == L.DOT_EINVAL
    assert lib.dot_mse_grad(None, None, None, -1, None, None, None) == L.DOT_EINVAL
    assert lib.dot_mse_grad(None, None, None, 5, None, None, None) == L.DOT_EINVAL
    assert lib.dot_mse_grad(None, None, None, 0, None, None, None) == L.DOT_OK
    assert lib.dot_gather_rows(None, 3, 10, None, None) == L.DOT_EINVAL
    assert b"power of two" in lib.dot_last_error()
    assert lib.dot_gather_rows(None, 4, 10, None, None) == L.DOT_EINVAL
    assert lib.dot_atomic_count(None, 8, -1, 0, None) == L.DOT_EINVAL
    assert lib.dot_atomic_count(None, 8, 5, 1, None) == L.DOT_EINVAL
    assert lib.dot_atomic_count(16, 0, 5, 0, None) == L.DOT_EINVAL
    assert lib.dot_atomic_count(None, 0, 0, 0, None) == L.DOT_OK
    assert lib.dot_pixel_batch(None, -1, 4, 4, 1, None, None, None, None, 0, None) == L.DOT_EINVAL
    assert lib.dot_pixel_batch(None, 4, 0, 4, 1, None, None, None, None, 0, None) == L.DOT_EINVAL
    assert lib.dot_pixel_batch(None, 4, 4, 4, 1, None, None, None, None, 0, None) == L.DOT_EINVAL
    assert lib.dot_pixel_batch(None, 4, 70000, 70000, 1, None, None, None, None, 0, None) == L.DOT_EINVAL
    assert b"2^31" in lib.dot_last_error()
    assert lib.dot_pixel_batch(None, 0, 4, 4, 1, None, None, None, None, 0, None) == L.DOT_OK
    # a sparser batch uses larger tiles (each holds ~64 of its rays), hence fewer bins
    w_dense = lib.dot_pixel_batch_workspace(1 << 20, 800, 800, 2)
    w_sparse = lib.dot_pixel_batch_workspace(1 << 10, 800, 800, 2)
    assert 0 < w_sparse < w_dense
    assert lib.dot_pixel_batch_workspace(4, 4, 4, 0) == 0


def test_noalloc_pixel_batch_argument_checks_need_no_device():
    """The no-allocation pixel batch refuses, before any device work, what
    dot_pixel_batch refuses and a batch whose scratch exceeds the array the
    library holds (pointers here are stand-ins that are never dereferenced)."""
    lib = L.load()
    fake = C.c_void_p(256)
    assert lib.dot_pixel_batch_noalloc(None, -1, 4, 4, 1, None, None, None, None) == L.DOT_EINVAL
    assert lib.dot_pixel_batch_noalloc(None, 4, 0, 4, 1, None, None, None, None) == L.DOT_EINVAL
    assert lib.dot_pixel_batch_noalloc(None, 4, 4, 4, 1, None, None, None, None) == L.DOT_EINVAL
    assert b"NULL" in lib.dot_last_error()
    assert lib.dot_pixel_batch_noalloc(None, 0, 4, 4, 1, None, None, None, None) == L.DOT_OK
    n = 4_000_000
    assert lib.dot_pixel_batch_workspace(n, 800, 800, 100) > (16 << 20)
    assert lib.dot_pixel_batch_noalloc(fake, n, 800, 800, 100, fake, fake, None, None) == L.DOT_EINVAL
    assert b"scratch" in lib.dot_last_error()


def test_serving_queue_argument_checks_need_no_device():
    """The persistent serving queue refuses malformed arguments before it
    allocates or launches anything."""
    lib = L.load()
    h = C.c_void_p()
    assert lib.dot_serve_open(7, 16, 1.0, None, C.byref(h)) == L.DOT_EINVAL
    assert lib.dot_serve_open(L.DOT_F16, 0, 1.0, None, C.byref(h)) == L.DOT_EINVAL
    assert lib.dot_serve_open(L.DOT_F16, 5000, 1.0, None, C.byref(h)) == L.DOT_EINVAL
    assert lib.dot_serve_open(L.DOT_F16, 16, 0.0, None, C.byref(h)) == L.DOT_EINVAL
    assert lib.dot_serve_open(L.DOT_F16, 16, float("inf"), None, C.byref(h)) == L.DOT_EINVAL
    assert lib.dot_serve_open(L.DOT_F16, 16, 1.0, None, None) == L.DOT_EINVAL
    t = C.c_int64()
    assert lib.dot_serve_push(None, None, C.byref(t)) == L.DOT_EINVAL
    assert lib.dot_serve_done(None, 0) == L.DOT_EINVAL
    assert lib.dot_serve_close(None) == L.DOT_OK
