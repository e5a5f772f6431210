"""FP64 oracle of the median-cut quantisation of the SH coefficients.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; the product path never
imports it.

The paper compresses its octrees by quantising the SH coefficients with
Heckbert's median-cut algorithm (Sec. 4.1, "Compression"; the starred rows of
Tab. S1 and Tab. S2).  It gives no further detail, so this module fixes one
reading and implements it plainly:

  * the quantised vector is the whole SH row of a leaf (3 K values, as
    stored), so a leaf keeps one palette index;
  * median cut in rounds: every box of the current round is split, so after
    ``bits`` rounds there are 2^bits boxes (some may be empty when there are
    few leaves);
  * a box is split along its widest dimension -- the largest max - min over
    its members (ties: the lowest dimension) -- at the median: its members
    ordered by their value in that dimension (ties: lower leaf index) go
    ``n // 2`` to the lower box (index 2b) and the rest to the upper box
    (2b + 1); -0.0 and +0.0 compare equal;
  * the palette entry of a box is the mean of its members' rows (FP64, rounded
    once to the palette's storage type); an empty box's entry is zero.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def median_cut(X, bits):
    """X: [N, D] leaf rows (values as stored).  Returns (index int64 [N],
    palette float64 [2^bits, D] unrounded means, counts int64 [2^bits])."""
    X = np.asarray(X, np.float64)
    N, D = X.shape
    box = np.zeros(N, np.int64)
    leaf = np.arange(N)
    for r in range(bits):
        new = np.empty(N, np.int64)
        order = np.argsort(box, kind="stable")          # members of each box, in leaf order
        starts = np.searchsorted(box[order], np.arange(2 ** r + 1))
        for b in range(2 ** r):
            m = order[starts[b]:starts[b + 1]]
            n = m.shape[0]
            if n == 0:
                continue
            V = X[m]
            width = V.max(axis=0) - V.min(axis=0)
            dim = int(np.argmax(width))                 # first of the widest
            rank = np.lexsort((leaf[m], V[:, dim]))     # by value, then by leaf index
            new[m[rank[:n // 2]]] = 2 * b
            new[m[rank[n // 2:]]] = 2 * b + 1
        box = new
    P = 2 ** bits
    counts = np.bincount(box, minlength=P)
    palette = np.zeros((P, D))
    np.add.at(palette, box, X)
    nz = counts > 0
    palette[nz] /= counts[nz, None]
    return box, palette, counts


def quantize_tree(sigma, sh, bits, storage="f16"):
    """The compressed leaf payload: (sigma rounded to `storage`, index [L],
    palette [2^bits, 3, K] rounded to `storage`, decoded sh [L, 3, K])."""
    sh = np.asarray(sh, np.float64)
    L = sh.shape[0]
    idx, pal, _ = median_cut(sh.reshape(L, -1), bits)
    pal = O.round_storage(pal, storage).reshape((2 ** bits,) + sh.shape[1:])
    sig = O.round_storage(np.asarray(sigma, np.float64), storage)
    return sig, idx, pal, pal[idx]
