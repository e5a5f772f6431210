"""Seeded synthetic inputs: SDF-driven octrees, leaf values and camera rigs.

This module produces *inputs* only.  It holds none of the renderer's arithmetic
(no ray generation, no spherical harmonics, no compositing, no refinement): both
the HIP library and the FP64 oracle consume what it returns and do their own
work on it.

The scenes stand in for the paper's datasets (NeRF-synthetic 800x800 with 100
training views, Tanks & Temples 1920x1080; Sec. 4.1), which are not available:
an octree over the root cube [-1,1]^3 is grown around the zero set of a signed
distance function, in place of the octree the paper resamples from a pretrained
NeRF-SH.  Leaves carry a density that peaks on the surface and random SH
coefficients (degree 2 or 3; Sec. 4.1 uses 16 coefficients per channel).

Canonical tree format (what ``dot_build`` and the oracle both accept):

* ``child``  int32 [n_internal, 8].  Octant ``o = x | y<<1 | z<<2`` (bit set =
  upper half along that axis).  Entry ``>= 0`` is an internal node index,
  entry ``< 0`` encodes leaf ``-1 - entry``.  Node 0 is the root.  A tree whose
  root is a leaf has ``n_internal == 0``.
* Internal nodes are numbered in depth-first pre-order, leaves in depth-first
  order (children visited in octant order), i.e. leaves are in Morton order.
* ``sigma`` [L], ``sh`` [L, 3, K] with K = (degree+1)^2.

Build rule: a node of depth d < D is subdivided iff |sdf(centre)| < 2 h_d,
where h_d = 2 / 2^d is its edge length.  Leaf density
sigma = 50 exp(-(sdf/0.05)^2) evaluated at the leaf centre in FP64; SH DC
coefficients ~ U(0,1), higher ones ~ N(0, 0.1^2); the DC array [L,3] is drawn
first, then the higher-order array [L,3,K-1], leaves in DFS order.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_CHUNK = 1 << 20


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(fn, n, out):
    """out[s:e] = fn(s, e) over chunks, on a thread pool (NumPy releases the GIL)."""
    spans = [(a, min(a + _CHUNK, n)) for a in range(0, n, _CHUNK)]

    def run(se):
        out[se[0]:se[1]] = fn(*se)

    if len(spans) <= 1:
        for se in spans:
            run(se)
    else:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(run, spans))
    return out

# ----------------------------------------------------------------------------
# Signed distance functions (FP64, vectorised over points [..., 3])
# ----------------------------------------------------------------------------


def sdf_sphere(radius=0.5, centre=(0.0, 0.0, 0.0)):
    c = np.asarray(centre, np.float64)

    def f(p):
        return np.linalg.norm(p - c, axis=-1) - radius

    return f


def sdf_torus_box(major=0.55, minor=0.18, half=0.3):
    """Union of a z-axis torus and an axis-aligned box, both at the origin."""

    def torus(p):
        q = np.sqrt(p[..., 0] ** 2 + p[..., 1] ** 2) - major
        return np.sqrt(q * q + p[..., 2] ** 2) - minor

    def box(p):
        q = np.abs(p) - half
        outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
        inside = np.minimum(np.max(q, axis=-1), 0.0)
        return outside + inside

    def f(p):
        return np.minimum(torus(p), box(p))

    return f


def sdf_terrain_ellipsoids(seed=2, n_ell=20, octaves=6, amp=0.12, base=-0.35, r_lo=0.04, r_hi=0.2):
    """Noisy height-field terrain (z below h(x,y) is solid) unioned with ellipsoids.

    The ellipsoid distance is the usual first-order estimate (|p/r| - 1) min r.
    """
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0, 2 * np.pi, octaves)
    phase = rng.uniform(0, 2 * np.pi, octaves)
    centres = rng.uniform(-0.8, 0.8, (n_ell, 3))
    radii = rng.uniform(r_lo, r_hi, (n_ell, 3))

    def height(x, y):
        h = np.full_like(x, base)
        for o in range(octaves):
            k = 2.0 ** (o + 1)
            h += amp * 2.0 ** (-o) * np.sin(
                k * (x * np.cos(theta[o]) + y * np.sin(theta[o])) + phase[o])
        return h

    def f(p):
        d = p[..., 2] - height(p[..., 0], p[..., 1])   # vertical distance to the surface
        for e in range(n_ell):
            q = (p - centres[e]) / radii[e]
            de = (np.linalg.norm(q, axis=-1) - 1.0) * radii[e].min()
            d = np.minimum(d, de)
        return d

    return f


# ----------------------------------------------------------------------------
# Morton helpers (used only to put generated nodes into DFS order)
# ----------------------------------------------------------------------------


def _spread3(v):
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton3(ijk):
    """Interleave integer coords [..., 3] -> uint64 (x in bit 0, y bit 1, z bit 2)."""
    ijk = np.asarray(ijk)
    return (_spread3(ijk[..., 0]) | (_spread3(ijk[..., 1]) << np.uint64(1))
            | (_spread3(ijk[..., 2]) << np.uint64(2)))


OCT = np.array([[o & 1, (o >> 1) & 1, (o >> 2) & 1] for o in range(8)], np.int64)


def tree_from_cells(leaf_depth, leaf_ijk, max_depth):
    """Canonical child array from a complete set of leaf cells.

    ``leaf_depth`` [L], ``leaf_ijk`` [L,3] (coords at the leaf's own depth) must
    tile the root cube.  Returns (child int32 [I,8], order) where ``order`` is
    the permutation that puts the given leaves into DFS order.
    """
    leaf_depth = np.asarray(leaf_depth, np.int64)
    leaf_ijk = np.asarray(leaf_ijk, np.int64)
    L = leaf_depth.shape[0]
    if L == 1:
        assert leaf_depth[0] == 0
        return np.zeros((0, 8), np.int32), np.zeros(1, np.int64)
    D = int(max_depth)
    shift = (D - leaf_depth)[:, None]
    lkey = morton3(leaf_ijk << shift)
    order = np.argsort(lkey, kind="stable")
    lkey = lkey[order]
    ld = leaf_depth[order]
    lijk = leaf_ijk[order]
    # every proper ancestor of every leaf is an internal node
    anc_d, anc_ijk = [], []
    for d in range(D):
        sel = ld > d
        if not sel.any():
            continue
        a = lijk[sel] >> (ld[sel] - d)[:, None]
        # unique per depth
        key = morton3(a)
        _, idx = np.unique(key, return_index=True)
        anc_ijk.append(a[idx])
        anc_d.append(np.full(idx.shape[0], d, np.int64))
    anc_d = np.concatenate(anc_d)
    anc_ijk = np.concatenate(anc_ijk)
    ikey = morton3(anc_ijk << (D - anc_d)[:, None])
    iorder = np.lexsort((anc_d, ikey))
    anc_d = anc_d[iorder]
    anc_ijk = anc_ijk[iorder]
    I = anc_d.shape[0]
    # node identity key: per-depth Morton code offset by depth so keys are unique
    off = np.array([sum(8 ** k for k in range(d)) for d in range(D + 2)], np.uint64)
    int_id = morton3(anc_ijk) + off[anc_d]
    leaf_id = morton3(lijk) + off[ld]
    int_sort = np.argsort(int_id)
    leaf_sort = np.argsort(leaf_id)
    child = np.empty((I, 8), np.int32)
    for o in range(8):
        cijk = anc_ijk * 2 + OCT[o]
        cid = morton3(cijk) + off[anc_d + 1]
        pos = np.searchsorted(int_id, cid, sorter=int_sort)
        pos = np.minimum(pos, I - 1)
        is_int = int_id[int_sort[pos]] == cid
        lpos = np.searchsorted(leaf_id, cid, sorter=leaf_sort)
        lpos = np.minimum(lpos, L - 1)
        is_leaf = leaf_id[leaf_sort[lpos]] == cid
        if not np.all(is_int ^ is_leaf):
            raise ValueError("leaf cells do not tile the root cube")
        child[:, o] = np.where(is_int, int_sort[pos], -1 - leaf_sort[lpos]).astype(np.int32)
    return child, order


# ----------------------------------------------------------------------------
# Scenes
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Scene:
    child: np.ndarray          # int32 [I, 8]
    leaf_depth: np.ndarray     # int32 [L]
    leaf_ijk: np.ndarray       # int64 [L, 3] coords at the leaf's own depth
    sigma64: np.ndarray        # float64 [L]   generator values
    sh32: np.ndarray           # float32 [L, 3, K] generator values (drawn in FP32)
    degree: int
    max_depth: int
    bbox_min: tuple = (-1.0, -1.0, -1.0)
    bbox_size: float = 2.0

    @property
    def n_leaves(self):
        return int(self.sigma64.shape[0])

    @property
    def n_internal(self):
        return int(self.child.shape[0])

    @property
    def sigma(self):
        return self.sigma64.astype(np.float32)

    @property
    def sh(self):
        return self.sh32

    @property
    def sh64(self):
        return self.sh32.astype(np.float64)


def grow_levels(split_fn, max_depth):
    """Grow an octree level by level.

    ``split_fn(d, ijk)`` returns a bool mask of the depth-d nodes to subdivide.
    Returns the per-level lists (coords [n_d,3], split mask [n_d]); the children
    of the j-th split node of level d are entries 8j..8j+7 of level d+1.
    """
    cur = np.zeros((1, 3), np.int64)
    levels = []
    for d in range(max_depth + 1):
        if d < max_depth and cur.shape[0]:
            split = np.asarray(split_fn(d, cur), bool)
        else:
            split = np.zeros(cur.shape[0], bool)
        levels.append((cur, split))
        par = cur[split]
        if par.shape[0] == 0:
            break
        cur = (par[:, None, :] * 2 + OCT[None, :, :]).reshape(-1, 3)
    return levels


def tree_from_levels(levels):
    """Canonical (DFS-numbered) child array and leaf list from grown levels.

    Returns (child int32 [I,8], leaf_depth int64 [L], leaf_ijk int64 [L,3]).
    """
    D = len(levels) - 1
    # breadth-first numbering: per level, internal and leaf ranks
    int_base, leaf_base = [], []
    ni = nl = 0
    for cur, split in levels:
        int_base.append(ni)
        leaf_base.append(nl)
        ni += int(split.sum())
        nl += int((~split).sum())
    I, L = ni, nl
    if I == 0:
        return (np.zeros((0, 8), np.int32), np.zeros(1, np.int64), np.zeros((1, 3), np.int64))
    # DFS ranks: internal nodes by (Morton of min corner at depth D, depth); leaves by Morton
    ikey, idep, lkey = [], [], []
    leaf_d, leaf_ijk = [], []
    for d, (cur, split) in enumerate(levels):
        c_int = cur[split]
        c_leaf = cur[~split]
        ikey.append(morton3(c_int << (D - d)))
        idep.append(np.full(c_int.shape[0], d, np.int64))
        lkey.append(morton3(c_leaf << (D - d)))
        leaf_d.append(np.full(c_leaf.shape[0], d, np.int64))
        leaf_ijk.append(c_leaf)
    ikey = np.concatenate(ikey)
    idep = np.concatenate(idep)
    lkey = np.concatenate(lkey)
    iorder = np.lexsort((idep, ikey))        # DFS position -> BFS index
    lorder = np.argsort(lkey, kind="stable")
    irank = np.empty(I, np.int64)
    irank[iorder] = np.arange(I)
    lrank = np.empty(L, np.int64)
    lrank[lorder] = np.arange(L)
    child = np.empty((I, 8), np.int32)
    for d in range(D):
        cur, split = levels[d]
        n_split = int(split.sum())
        if n_split == 0:
            continue
        nxt_cur, nxt_split = levels[d + 1]
        # BFS internal / leaf index of every child entry on level d+1
        is_int = nxt_split
        int_idx = int_base[d + 1] + np.cumsum(is_int) - 1
        leaf_idx = leaf_base[d + 1] + np.cumsum(~is_int) - 1
        val = np.where(is_int, irank[np.maximum(int_idx, 0)],
                       -1 - lrank[np.maximum(leaf_idx, 0)])
        parents = irank[int_base[d] + np.arange(n_split)]
        child[parents] = val.reshape(n_split, 8).astype(np.int32)
    leaf_d = np.concatenate(leaf_d)[lorder]
    leaf_ijk = np.concatenate(leaf_ijk)[lorder]
    return child, leaf_d, leaf_ijk


def _sdf_split(sdf, bbox_min, size, factor=2.0):
    bmin = np.asarray(bbox_min, np.float64)

    def split(d, ijk):
        h = size / 2.0 ** d
        out = np.empty(ijk.shape[0], bool)
        return _chunked(lambda a, b: np.abs(sdf(bmin + (ijk[a:b] + 0.5) * h)) < factor * h, ijk.shape[0], out)

    return split


def _random_sh(L, degree, rng, dc_lo=0.0, dc_hi=1.0, std=0.1):
    """SH coefficients drawn directly in FP32 (the generator values are exactly
    these FP32 numbers, so FP32 storage is lossless for SH).  Leaves are drawn
    in chunks of 2^20 from independent streams spawned from `rng` (chunk order
    fixed), DC first then the higher orders within each chunk."""
    K = (degree + 1) ** 2
    sh = np.empty((L, 3, K), np.float32)
    n_chunks = (L + _CHUNK - 1) // _CHUNK
    seeds = rng.bit_generator.seed_seq.spawn(n_chunks) if n_chunks else []

    def fill(a, b):
        r = np.random.default_rng(seeds[a // _CHUNK])
        blk = np.empty((b - a, 3, K), np.float32)
        blk[:, :, 0] = np.float32(dc_lo) + np.float32(dc_hi - dc_lo) * r.random((b - a, 3), dtype=np.float32)
        if K > 1:
            hi = r.standard_normal((b - a, 3, K - 1), dtype=np.float32)
            hi *= np.float32(std)
            blk[:, :, 1:] = hi
        return blk

    return _chunked(fill, L, sh)


def make_scene(sdf, max_depth, degree, seed, sigma_peak=50.0, shell=0.05,
               bbox_min=(-1.0, -1.0, -1.0), size=2.0):
    levels = grow_levels(_sdf_split(sdf, bbox_min, size), max_depth)
    child, ld, lijk = tree_from_levels(levels)
    h = size / 2.0 ** ld
    L = ld.shape[0]
    sigma = np.empty(L, np.float64)
    bmin = np.asarray(bbox_min, np.float64)
    _chunked(lambda a, b: sigma_peak * np.exp(-(sdf(bmin + (lijk[a:b] + 0.5) * h[a:b, None]) / shell) ** 2),
             L, sigma)
    rng = np.random.default_rng(seed)
    sh = _random_sh(L, degree, rng)
    return Scene(child=child, leaf_depth=ld.astype(np.int32), leaf_ijk=lijk,
                 sigma64=sigma, sh32=sh, degree=degree, max_depth=max_depth,
                 bbox_min=tuple(bbox_min), bbox_size=size)


def uniform_scene(depth, degree, sigma, sh_dc=0.0, seed=None):
    """Depth-uniform tree (8^depth leaves) with constant or random values."""
    levels = grow_levels(lambda d, ijk: np.ones(ijk.shape[0], bool), depth)
    child, ld, lijk = tree_from_levels(levels)
    L = ld.shape[0]
    K = (degree + 1) ** 2
    if seed is None:
        sig = np.full(L, float(sigma))
        sh = np.zeros((L, 3, K), np.float32)
        sh[:, :, 0] = sh_dc
    else:
        rng = np.random.default_rng(seed)
        sig = rng.uniform(0.0, float(sigma), L)
        sh = _random_sh(L, degree, rng, 0.0, 1.0, 0.3)
    return Scene(child=child, leaf_depth=ld.astype(np.int32), leaf_ijk=lijk,
                 sigma64=sig, sh32=sh, degree=degree, max_depth=depth)


def random_tree_scene(max_depth, degree, seed, p_split=0.45, sigma_max=8.0):
    """Random-topology tree: the root splits, deeper nodes split with probability p_split."""
    rng = np.random.default_rng(seed)

    def split(d, ijk):
        if d == 0:
            return np.ones(ijk.shape[0], bool)
        return rng.random(ijk.shape[0]) < p_split

    levels = grow_levels(split, max_depth)
    child, ld, lijk = tree_from_levels(levels)
    L = ld.shape[0]
    sig = rng.uniform(0.0, sigma_max, L)
    sh = _random_sh(L, degree, rng, -1.0, 1.0, 0.3)
    return Scene(child=child, leaf_depth=ld.astype(np.int32), leaf_ijk=lijk,
                 sigma64=sig, sh32=sh, degree=degree, max_depth=max_depth)


# ----------------------------------------------------------------------------
# Cameras.  A camera is (c2w[3x4] row-major, fx, fy, cx, cy, width, height):
# camera axes x right, y down, z forward; world = R @ cam + t.
# ----------------------------------------------------------------------------

CAMERA_DTYPE = np.dtype([("c2w", np.float32, (12,)), ("fx", np.float32), ("fy", np.float32),
                         ("cx", np.float32), ("cy", np.float32),
                         ("width", np.int32), ("height", np.int32)])


def look_at_camera(az_deg, el_deg, radius, width, height, fov_deg=40.0):
    az, el = math.radians(az_deg), math.radians(el_deg)
    pos = radius * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az),
                             math.sin(el)])
    return _camera_at(pos, width, height, fov_deg)


def _camera_at(pos, width, height, fov_deg):
    pos = np.asarray(pos, np.float64)
    fwd = -pos / np.linalg.norm(pos)
    up = np.array([0.0, 0.0, 1.0])
    if abs(fwd @ up) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd], axis=1)
    cam = np.zeros((), CAMERA_DTYPE)
    cam["c2w"] = np.concatenate([R, pos[:, None]], axis=1).reshape(-1)
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    cam["fx"] = f
    cam["fy"] = f
    cam["cx"] = width / 2.0
    cam["cy"] = height / 2.0
    cam["width"] = width
    cam["height"] = height
    return cam


def cameras(specs):
    arr = np.zeros(len(specs), CAMERA_DTYPE)
    for i, s in enumerate(specs):
        arr[i] = look_at_camera(*s)
    return arr


def random_sphere_cameras(n, radius, width, height, seed, fov_deg=40.0):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    arr = np.zeros(n, CAMERA_DTYPE)
    for i in range(n):
        arr[i] = _camera_at(radius * v[i], width, height, fov_deg)
    return arr


def random_explicit_rays(n, seed, radius=3.0, spread=1.0):
    """Random rays aimed at the root cube: origin on a sphere, target inside it."""
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o *= radius / np.linalg.norm(o, axis=1, keepdims=True)
    tgt = rng.uniform(-spread, spread, (n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


# ----------------------------------------------------------------------------
# The workloads
# ----------------------------------------------------------------------------


def sphere_scene():
    """Sphere r=0.5, depth 5, degree 2, seed 0."""
    return make_scene(sdf_sphere(0.5), max_depth=5, degree=2, seed=0)


def sphere_camera():
    """One 64x64 camera at radius 4, azimuth 30, elevation 20, 40 deg FOV."""
    return cameras([(30.0, 20.0, 4.0, 64, 64)])


def torus_box_scene():
    """Torus (R=0.55, r=0.18) union box (half 0.3), depth 9, degree 3, seed 1."""
    return make_scene(sdf_torus_box(), max_depth=9, degree=3, seed=1)


def ring_cameras(width=800, height=800):
    """Eight views on the radius-4 sphere: azimuth 45j, elevation +-30 alternating."""
    return cameras([(45.0 * j, 30.0 if j % 2 == 0 else -30.0, 4.0, width, height)
                    for j in range(8)])


def sphere_views(n=100, width=800, height=800, seed=11):
    return random_sphere_cameras(n, 4.0, width, height, seed)


def terrain_scene():
    """Terrain + 20 ellipsoids, depth 10, degree 3, seed 2."""
    return make_scene(sdf_terrain_ellipsoids(seed=2), max_depth=10, degree=3, seed=2)


def terrain_cameras(width=1920, height=1080):
    return cameras([(90.0 * j + 20.0, 25.0, 4.0, width, height) for j in range(4)])


def training_views(n=100, size=64, seed=3):
    return random_sphere_cameras(n, 4.0, size, size, seed + 100)


def perturb_sh(scene, std=0.05, seed=3):
    """Training copy: SH + N(0, std^2), sigma unperturbed."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(scene.sh32.shape, dtype=np.float32) * np.float32(std)
    return dataclasses.replace(scene, sh32=scene.sh32 + noise)


def ray_permutations(n_rays, epochs, seed):
    """One random order of the training rays per epoch (the permutation step of
    the training loop), drawn from a seeded generator."""
    rng = np.random.default_rng(seed)
    return [rng.permutation(n_rays).astype(np.int64) for _ in range(epochs)]


def pixel_batch(n_views, width, height, batch, seed):
    """Random (view, pixel) pairs without replacement from the view pool."""
    rng = np.random.default_rng(seed)
    pool = n_views * width * height
    idx = rng.permutation(pool)[:batch]
    cam = (idx // (width * height)).astype(np.int32)
    pix = (idx % (width * height)).astype(np.int32)
    return cam, pix
