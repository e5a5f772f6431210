"""The no-allocation pixel batch (dot_pixel_batch_noalloc, scratch in a
device array the library holds) against dot_pixel_batch with a caller
workspace, through the C ABI: two calls in a row, the second on a smaller
batch (the array keeps the first call's contents), on the many-tile path
(one atomic per ray) and the few-tile path (LDS histograms).  The order of
rays inside a screen tile is left to scheduling, so each output position's
camera and tile must agree and each tile must hold the same rays; the
batch's content must be the input's."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _tile_shift(n, W, H, n_cams):
    # the documented tile size: square, 8..128 px, the smallest holding about 16 of the batch's rays
    density = n / (n_cams * W * H)
    s = 3
    while s < 7 and (1 << (2 * s)) * density < 16.0:
        s += 1
    return s


def _tiles(cam, pix, W, H, shift):
    tw = (W + (1 << shift) - 1) >> shift
    th = (H + (1 << shift) - 1) >> shift
    v, u = pix // W, pix % W
    return cam.astype(np.int64) * tw * th + (v >> shift) * tw + (u >> shift)


def _run(lib, L, ids, W, H, n_cams, noalloc):
    from paper_2307_15333_amd import core
    n = ids.shape[0]
    cam = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    pix = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    out = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    args = [C.c_void_p(ids.data_ptr()), C.c_int64(n), W, H, n_cams, C.c_void_p(cam.data_ptr()),
            C.c_void_p(pix.data_ptr()), C.c_void_p(out.data_ptr())]
    if noalloc:
        L.check(lib.dot_pixel_batch_noalloc(*args, core._stream()))
    else:
        need = lib.dot_pixel_batch_workspace(n, W, H, n_cams)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        L.check(lib.dot_pixel_batch(*args, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()), core._stream()))
    torch.cuda.synchronize()
    return cam.cpu().numpy(), pix.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("W,H,n_cams,sizes", [(800, 800, 100, (1 << 20, 300_001)),   # many tiles
                                              (64, 64, 100, (1 << 18, 70_001))])      # at most 4096 tiles
def test_noalloc_pixel_batch_matches_workspace_entry_point(W, H, n_cams, sizes):
    from paper_2307_15333_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(11)
    for n in sizes:
        print(f"noalloc pixel batch: {n} rays of {n_cams} views at {W}x{H}", flush=True)
        ids_np = rng.choice(n_cams * W * H, n, replace=False).astype(np.int64)
        ids = torch.as_tensor(ids_np, device="cuda")
        ca, pa, oa = _run(lib, L, ids, W, H, n_cams, noalloc=False)
        cb, pb, ob = _run(lib, L, ids, W, H, n_cams, noalloc=True)
        # the batch's content is the input's, and each output is consistent with its id
        np.testing.assert_array_equal(np.sort(ob), np.sort(ids_np))
        np.testing.assert_array_equal(cb.astype(np.int64) * W * H + pb, ob)
        np.testing.assert_array_equal(ca.astype(np.int64) * W * H + pa, oa)
        # position by position the same camera and tile; within a tile the same rays
        shift = _tile_shift(n, W, H, n_cams)
        ta, tb = _tiles(ca, pa, W, H, shift), _tiles(cb, pb, W, H, shift)
        np.testing.assert_array_equal(ca, cb)
        np.testing.assert_array_equal(ta, tb)
        assert np.all(np.diff(tb) >= 0)
        key_a = np.lexsort((oa, ta))
        key_b = np.lexsort((ob, tb))
        np.testing.assert_array_equal(oa[key_a], ob[key_b])


def test_noalloc_pixel_batch_rejects_a_batch_beyond_its_scratch():
    from paper_2307_15333_amd import _lib as L
    lib = L.load()
    n = 4_000_000
    assert lib.dot_pixel_batch_workspace(n, 800, 800, 100) > (16 << 20)
    ids = torch.zeros(n, dtype=torch.int64, device="cuda")
    o32 = torch.empty(n, dtype=torch.int32, device="cuda")
    rc = lib.dot_pixel_batch_noalloc(C.c_void_p(ids.data_ptr()), C.c_int64(n), 800, 800, 100,
                                     C.c_void_p(o32.data_ptr()), C.c_void_p(o32.data_ptr()), None, None)
    assert rc == L.DOT_EINVAL
    assert b"scratch" in lib.dot_last_error()
