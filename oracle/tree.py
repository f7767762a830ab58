"""Octree of the multilevel FMM (TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).

Section 2 defines the boxes B^l_alpha of side a_l (root l = 0, highest active level l = 2), the
neighbour list N(B) (B and the boxes adjacent to it) and the interaction list I(B): the boxes of
the same level that are not neighbours of B but whose parent neighbours the parent of B.
Section 3.2 counts 316 distinct transfer vectors per level, which fixes "adjacent" as
"Chebyshev distance <= 1 in box units" (7^3 - 3^3 = 316 offsets).

Readings of what the paper leaves open:
* Root cube: corner lo = per-axis minimum of the points, side S = largest per-axis extent (S = 1
  if every point coincides).
* Leaf index per axis: min(floor((x - lo) * (2^L / S)), 2^L - 1), in FP64, with the factor
  2^L / S computed first.
* Morton key: bit b of the x index goes to bit 3b, of y to 3b + 1, of z to 3b + 2. Points are
  stably sorted by their key at the finest resolution, 21 bits per axis (ties keep the input
  order); the key of a depth-L leaf is that key shifted right by 3 (21 - L) bits. Because the
  factor 2^21 / S is 2^(21 - L) times 2^L / S exactly, the shifted fine index equals the depth-L
  index above.
* Only occupied boxes exist; empty boxes contribute nothing to any sum.
* Depth (when not given): the smallest L >= 2 whose fullest leaf holds <= max_leaf points.
* List order: every neighbour / interaction list is sorted by source box index (Morton order).
"""
import numpy as np


MAX_DEPTH = 21


def root_cube(x):
    """Root cube corner and side (reading above)."""
    lo = x.min(axis=0)
    ext = x.max(axis=0) - lo
    side = float(ext.max())
    if side == 0.0:
        side = 1.0
    return lo, side


def quantize(x, lo, side, depth):
    """Leaf index per axis (reading above)."""
    scale = float(2 ** depth) / side
    t = (x - lo[None, :]) * scale
    idx = np.floor(t).astype(np.int64)
    return np.minimum(idx, 2 ** depth - 1)


def morton(idx, depth):
    """Interleave the per-axis indices (reading above)."""
    key = np.zeros(idx.shape[0], dtype=np.uint64)
    for b in range(depth):
        for a in range(3):
            bit = (idx[:, a] >> b) & 1
            key |= bit.astype(np.uint64) << np.uint64(3 * b + a)
    return key


def demorton(key, nbits):
    """Per-axis indices of Morton keys with nbits bits per axis."""
    idx = np.zeros((key.shape[0], 3), dtype=np.int64)
    for b in range(nbits):
        for a in range(3):
            idx[:, a] |= ((key >> np.uint64(3 * b + a)) & np.uint64(1)).astype(np.int64) << b
    return idx


def auto_depth(x, max_leaf, max_depth=21):
    """Smallest L >= 2 whose fullest leaf holds <= max_leaf points (reading above)."""
    lo, side = root_cube(x)
    for depth in range(2, max_depth + 1):
        key = morton(quantize(x, lo, side, depth), depth)
        _, counts = np.unique(key, return_counts=True)
        if counts.max() <= max_leaf:
            return depth
    return max_depth


class Level:
    """Occupied boxes of one level: sorted Morton keys, integer coordinates, centres."""

    def __init__(self, keys, l, lo, side):
        self.l = l
        self.keys = keys
        self.ijk = demorton(keys, l)
        self.a = side / 2 ** l
        self.centers = lo[None, :] + (self.ijk + 0.5) * self.a
        self.n = len(keys)

    def find(self, ijk):
        """Index of the box with integer coordinates ijk [..., 3] (-1 if not occupied)."""
        ijk = np.asarray(ijk)
        inside = np.all((ijk >= 0) & (ijk < 2 ** self.l), axis=-1)
        safe = np.where(inside[..., None], ijk, 0)
        k = morton(safe.reshape(-1, 3), self.l).reshape(ijk.shape[:-1])
        pos = np.searchsorted(self.keys, k)
        pos = np.minimum(pos, self.n - 1)
        hit = inside & (self.keys[pos] == k)
        return np.where(hit, pos, -1)


def _csr(rows_lists):
    ptr = np.zeros(len(rows_lists) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows_lists])
    data = np.concatenate(rows_lists) if len(rows_lists) else np.zeros(0, np.int64)
    return ptr, data.astype(np.int64)


OFFS27 = np.array([(i, j, k) for k in (-1, 0, 1) for j in (-1, 0, 1) for i in (-1, 0, 1)],
                  dtype=np.int64)
OCT8 = np.array([(i, j, k) for k in (0, 1) for j in (0, 1) for i in (0, 1)], dtype=np.int64)


def offset_code(d):
    """Code 0..342 of a transfer offset d in [-3, 3]^3 (in box units): (dx+3) + 7 (dy+3) + 49 (dz+3)."""
    d = np.asarray(d)
    return (d[..., 0] + 3) + 7 * (d[..., 1] + 3) + 49 * (d[..., 2] + 3)


class Tree:
    """Octree with levels 0..depth over sorted points (Section 2)."""

    def __init__(self, x, depth=None, max_leaf=64):
        x = np.ascontiguousarray(x, dtype=np.float64)
        self.n = x.shape[0]
        if depth is None:
            depth = auto_depth(x, max_leaf)
        self.depth = depth
        self.lo, self.side = root_cube(x)
        self.idx = quantize(x, self.lo, self.side, depth)
        self.leaf_key = morton(self.idx, depth)
        self.fine_key = morton(quantize(x, self.lo, self.side, MAX_DEPTH), MAX_DEPTH)
        assert np.array_equal(self.fine_key >> np.uint64(3 * (MAX_DEPTH - depth)), self.leaf_key)
        self.perm = np.argsort(self.fine_key, kind="stable")
        self.sorted_keys = self.leaf_key[self.perm]
        self.xs = x[self.perm]
        self.levels = {}
        for l in range(depth, -1, -1):
            k = self.sorted_keys >> np.uint64(3 * (depth - l))
            self.levels[l] = Level(np.unique(k), l, self.lo, self.side)
        leaf = self.levels[depth]
        self.point_box = np.searchsorted(leaf.keys, self.sorted_keys)
        self.leaf_start = np.searchsorted(self.sorted_keys, leaf.keys, side="left")
        self.leaf_count = np.searchsorted(self.sorted_keys, leaf.keys, side="right") - self.leaf_start
        self.parent = {}
        for l in range(1, depth + 1):
            pk = self.levels[l].keys >> np.uint64(3)
            self.parent[l] = np.searchsorted(self.levels[l - 1].keys, pk)
        self.neighbors = {}
        self.ilist = {}
        self.ioff = {}
        for l in range(2, depth + 1):
            self.neighbors[l] = self._neighbors(l)
            self.ilist[l], self.ioff[l] = self._interaction(l)

    def _neighbors(self, l):
        """N(B): occupied boxes at Chebyshev distance <= 1, B included, sorted (Section 2)."""
        lev = self.levels[l]
        cand = lev.find(lev.ijk[:, None, :] + OFFS27[None, :, :])
        rows = [np.sort(c[c >= 0]) for c in cand]
        return _csr(rows)

    def _interaction(self, l):
        """I(B): children of the parent's neighbours that are not neighbours of B (Section 2).
        Also returns the offset code of each entry (source minus target, box units)."""
        lev = self.levels[l]
        par = self.levels[l - 1]
        pijk = par.ijk[self.parent[l]]                                   # [n, 3]
        cand_par = pijk[:, None, :] + OFFS27[None, :, :]                 # [n, 27, 3]
        child = 2 * cand_par[:, :, None, :] + OCT8[None, None, :, :]      # [n, 27, 8, 3]
        child = child.reshape(lev.n, 216, 3)
        d = child - lev.ijk[:, None, :]
        far = np.max(np.abs(d), axis=-1) > 1
        idx = lev.find(child)
        ok = far & (idx >= 0)
        rows, offs = [], []
        for b in range(lev.n):
            s = idx[b][ok[b]]
            o = offset_code(d[b][ok[b]])
            order = np.argsort(s)
            rows.append(s[order])
            offs.append(o[order])
        ptr, data = _csr(rows)
        _, odata = _csr(offs)
        return (ptr, data), odata
