"""Independent helpers used by the oracle pins (pure Python / NumPy).

These are textbook algorithms written separately from the oracle, so that an
error in the oracle shows up as a disagreement: a slab chord length, a 3D-DDA
grid walk (Amanatides & Woo 1987), point location by descending the child
array, and a leaf-list refinement built through the input generator's tree
constructor.
"""
import numpy as np

from paper_2307_15333_amd import synth


def slab_chord(o, d, lo=-1.0, hi=1.0):
    """(t_in, t_out) of the ray o + t d (t >= 0) in the cube [lo, hi]^3, or None."""
    t0, t1 = 0.0, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if not (lo <= o[a] <= hi):
                return None
            continue
        ta, tb = (lo - o[a]) / d[a], (hi - o[a]) / d[a]
        ta, tb = min(ta, tb), max(ta, tb)
        t0, t1 = max(t0, ta), min(t1, tb)
    return (t0, t1) if t0 < t1 else None


def dda_grid(o, d, n, lo=-1.0, size=2.0):
    """Cells (i,j,k) and lengths crossed by a unit-direction ray in an n^3 grid."""
    ch = slab_chord(o, d, lo, lo + size)
    if ch is None:
        return [], []
    t0, t1 = ch
    h = size / n
    p = o + t0 * d
    cell = np.clip(np.floor((p - lo) / h).astype(int), 0, n - 1)
    # the entry face fixes the coordinate along the entry axis
    step = np.where(d > 0, 1, -1)
    tmax = np.empty(3)
    tdelta = np.empty(3)
    for a in range(3):
        if d[a] == 0:
            tmax[a] = np.inf
            tdelta[a] = np.inf
        else:
            nxt = lo + (cell[a] + (1 if d[a] > 0 else 0)) * h
            tmax[a] = (nxt - o[a]) / d[a]
            tdelta[a] = h / abs(d[a])
    cells, lens = [], []
    t = t0
    while True:
        a = int(np.argmin(tmax))
        tn = min(tmax[a], t1)
        if tn > t:
            cells.append(tuple(cell))
            lens.append(tn - t)
        t = tn
        if t >= t1:
            break
        cell[a] += step[a]
        if cell[a] < 0 or cell[a] >= n:
            break
        tmax[a] += tdelta[a]
    return cells, lens


def locate_leaf(child, p, lo=-1.0, size=2.0):
    """Leaf id containing point p (descend the child array)."""
    if child.shape[0] == 0:
        return 0
    node = 0
    base = np.full(3, lo, np.float64)
    s = size
    while True:
        s /= 2
        oc = 0
        for a in range(3):
            if p[a] >= base[a] + s:
                oc |= 1 << a
                base[a] += s
        e = int(child[node, oc])
        if e < 0:
            return -1 - e
        node = e


def refine_by_leaf_list(scene, signal, tau, sample_frac, max_depth, prune_le=True):
    """Expected refined topology, computed on the leaf list (no child array walk):
    parents whose 8 leaf children are all selected become one leaf; the top-k
    eligible leaves become 8 leaves each.  Returns (child, depth, ijk, merged, k)."""
    ld = scene.leaf_depth.astype(np.int64)
    lijk = scene.leaf_ijk.astype(np.int64)
    L = ld.shape[0]
    s = np.asarray(signal, np.float64)
    sel = s <= tau if prune_le else s < tau
    # group leaves by parent cell
    groups = {}
    for i in range(L):
        if ld[i] == 0:
            continue
        key = (ld[i] - 1, tuple(lijk[i] >> 1))
        groups.setdefault(key, []).append(i)
    merged_parent = {}
    for key, mem in groups.items():
        if len(mem) == 8 and all(sel[m] for m in mem):
            merged_parent[key] = mem
    in_merge = np.zeros(L, bool)
    for mem in merged_parent.values():
        in_merge[mem] = True
    elig = np.where((~sel) & (ld < max_depth))[0]
    k = min(int(np.floor(sample_frac * L)), elig.shape[0])
    order = sorted(elig.tolist(), key=lambda i: (-s[i], i))
    split = set(order[:k])
    new_d, new_ijk = [], []
    for (d, pijk) in merged_parent:
        new_d.append(d)
        new_ijk.append(pijk)
    for i in range(L):
        if in_merge[i]:
            continue
        if i in split:
            for oc in range(8):
                new_d.append(ld[i] + 1)
                new_ijk.append(tuple(lijk[i] * 2 + synth.OCT[oc]))
        else:
            new_d.append(ld[i])
            new_ijk.append(tuple(lijk[i]))
    new_d = np.array(new_d, np.int64)
    new_ijk = np.array(new_ijk, np.int64)
    D = int(new_d.max())
    child, order = synth.tree_from_cells(new_d, new_ijk, max(D, 1))
    return child, new_d[order], new_ijk[order], len(merged_parent), k
