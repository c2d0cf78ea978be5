"""Uniform octree with locational (Morton) keys and pruned empty branches
(Section 2: a bounding box recursively subdivided into equal children; the
paper prunes branches that hold no points instead of refining adaptively;
Morton-ordered buffers are described in Appendix A.3).

Test infrastructure only (see ``oracle/__init__``).

Conventions the paper leaves open (shared with the library's header):

* Domain: a cube with lower corner ``origin`` and side ``width``.  A point x
  falls in the leaf with anchor a = min(floor((x - origin) / width * 2^d),
  2^d - 1) per axis; points outside the cube are rejected.
* Morton key of a box with anchor a at level l: the bits of a_x, a_y, a_z
  interleaved (bit b of a_x at position 3b, of a_y at 3b+1, of a_z at 3b+2)
  with a sentinel bit at position 3l, so parent = key >> 3 and the octant of
  a child is key & 7.
* Points are ordered by (leaf key, original index).
* Boxes at each level are the ancestors of non-empty leaves (of sources or
  targets), sorted by key.
* Near field of a leaf: leaves whose anchors differ by at most 1 in every
  axis, the leaf itself included (Section 2).
* Interaction list of a box at level l >= 2: boxes at level l whose parent is
  the box's parent or one of its neighbours, excluding the box's own near
  field (Section 2, the M2L bullet).  Sorted by source key.  The transfer
  vector t = a_source - a_target lies in [-3, 3]^3 with max |t_i| >= 2, and its
  index is its rank in lexicographic (t_x, t_y, t_z) order over those 316
  offsets (Section 3.1 counts them as 7^3 - 3^3).
"""

from __future__ import annotations

import itertools

import numpy as np

TRANSFER_VECTORS = np.array(
    [t for t in itertools.product(range(-3, 4), repeat=3) if max(abs(c) for c in t) >= 2],
    dtype=np.int64)
NEAR_OFFSETS = np.array(list(itertools.product(range(-1, 2), repeat=3)), dtype=np.int64)


def leaf_anchors(points: np.ndarray, origin, width: float, depth: int) -> np.ndarray:
    """Integer anchors of the depth-``depth`` leaves holding each point."""
    o = np.asarray(origin, dtype=np.float64)
    u = (points - o) / width
    if np.any(u < 0.0) or np.any(u > 1.0):
        raise ValueError("point outside the domain cube")
    a = np.floor(u * float(2 ** depth)).astype(np.int64)
    return np.minimum(a, 2 ** depth - 1)


def morton_keys(anchors: np.ndarray, level: int) -> np.ndarray:
    """Sentinel-bit Morton keys (uint64) of integer anchors (m, 3) at ``level``."""
    a = np.asarray(anchors, dtype=np.uint64)
    m = np.zeros(a.shape[0], dtype=np.uint64)
    one = np.uint64(1)
    for b in range(level):
        for ax in range(3):
            bit = (a[:, ax] >> np.uint64(b)) & one
            m |= bit << np.uint64(3 * b + ax)
    return m | (one << np.uint64(3 * level))


def key_anchors(keys: np.ndarray, level: int) -> np.ndarray:
    """Inverse of ``morton_keys``: anchors (m, 3) int64 of keys at ``level``."""
    k = np.asarray(keys, dtype=np.uint64)
    out = np.zeros((k.shape[0], 3), dtype=np.int64)
    one = np.uint64(1)
    for b in range(level):
        for ax in range(3):
            bit = (k >> np.uint64(3 * b + ax)) & one
            out[:, ax] |= bit.astype(np.int64) << b
    return out


def box_centers(keys: np.ndarray, level: int, origin, width: float) -> np.ndarray:
    """Centres of boxes at ``level``: origin + (a + 1/2) * width / 2^level."""
    w = width / 2 ** level
    return np.asarray(origin, dtype=np.float64) + (key_anchors(keys, level) + 0.5) * w


def transfer_index(t: np.ndarray) -> np.ndarray:
    """Lexicographic rank of offsets t (m, 3) among the 316 transfer vectors."""
    lut = -np.ones(7 ** 3, dtype=np.int64)
    code = (TRANSFER_VECTORS[:, 0] + 3) * 49 + (TRANSFER_VECTORS[:, 1] + 3) * 7 + (TRANSFER_VECTORS[:, 2] + 3)
    lut[code] = np.arange(len(TRANSFER_VECTORS))
    t = np.asarray(t, dtype=np.int64)
    return lut[(t[:, 0] + 3) * 49 + (t[:, 1] + 3) * 7 + (t[:, 2] + 3)]


class Tree:
    """Pruned uniform octree over sources and targets."""

    def __init__(self, sources: np.ndarray, targets: np.ndarray, depth: int,
                 origin=(0.0, 0.0, 0.0), width: float = 1.0):
        self.depth = int(depth)
        self.origin = np.asarray(origin, dtype=np.float64)
        self.width = float(width)
        self.sources = np.asarray(sources, dtype=np.float64)
        self.targets = np.asarray(targets, dtype=np.float64)
        d = self.depth
        sk = morton_keys(leaf_anchors(self.sources, origin, width, d), d)
        tk = morton_keys(leaf_anchors(self.targets, origin, width, d), d)
        self.src_perm = np.argsort(sk, kind="stable")
        self.tgt_perm = np.argsort(tk, kind="stable")
        self.src_keys_sorted = sk[self.src_perm]
        self.tgt_keys_sorted = tk[self.tgt_perm]
        leaves = np.union1d(np.unique(sk), np.unique(tk)).astype(np.uint64)
        self.levels = [None] * (d + 1)
        self.levels[d] = leaves
        for lev in range(d - 1, -1, -1):
            self.levels[lev] = np.unique(self.levels[lev + 1] >> np.uint64(3))
        self.src_start = np.searchsorted(self.src_keys_sorted, leaves, side="left")
        self.src_end = np.searchsorted(self.src_keys_sorted, leaves, side="right")
        self.tgt_start = np.searchsorted(self.tgt_keys_sorted, leaves, side="left")
        self.tgt_end = np.searchsorted(self.tgt_keys_sorted, leaves, side="right")

    def index_of(self, level: int, keys: np.ndarray) -> np.ndarray:
        """Position of ``keys`` in level ``level`` (-1 where absent)."""
        lv = self.levels[level]
        keys = np.asarray(keys, dtype=np.uint64)
        pos = np.searchsorted(lv, keys)
        pos_c = np.minimum(pos, len(lv) - 1)
        ok = (pos < len(lv)) & (lv[pos_c] == keys)
        return np.where(ok, pos_c, -1)

    def center(self, level: int, idx) -> np.ndarray:
        return box_centers(self.levels[level][idx], level, self.origin, self.width)

    def interactions(self, level: int):
        """CSR interaction lists at ``level`` (>= 2).

        Returns (offsets, source_index, t_index): targets are the boxes of the
        level in key order, each target's sources ascend by key.
        """
        if level < 2:
            raise ValueError("interaction lists start at level 2")
        keys = self.levels[level]
        a = key_anchors(keys, level)
        n = 2 ** level
        tg, sr, ti = [], [], []
        for it, t in enumerate(TRANSFER_VECTORS):
            c = a + t
            inside = np.all((c >= 0) & (c < n), axis=1)
            par_ok = np.max(np.abs((c >> 1) - (a >> 1)), axis=1) <= 1
            sel = np.nonzero(inside & par_ok)[0]
            if sel.size == 0:
                continue
            src = self.index_of(level, morton_keys(c[sel], level))
            ok = src >= 0
            tg.append(sel[ok])
            sr.append(src[ok])
            ti.append(np.full(int(ok.sum()), it, dtype=np.int64))
        if tg:
            tg = np.concatenate(tg)
            sr = np.concatenate(sr)
            ti = np.concatenate(ti)
        else:
            tg = sr = ti = np.zeros(0, dtype=np.int64)
        order = np.lexsort((sr, tg))
        tg, sr, ti = tg[order], sr[order], ti[order]
        offs = np.zeros(len(keys) + 1, dtype=np.int64)
        np.add.at(offs, tg + 1, 1)
        return np.cumsum(offs), sr, ti

    def near(self):
        """CSR near-field lists of the leaves (27-box neighbourhood, self included)."""
        d = self.depth
        keys = self.levels[d]
        a = key_anchors(keys, d)
        n = 2 ** d
        tg, sr = [], []
        for off in NEAR_OFFSETS:
            c = a + off
            inside = np.all((c >= 0) & (c < n), axis=1)
            sel = np.nonzero(inside)[0]
            src = self.index_of(d, morton_keys(c[sel], d))
            ok = src >= 0
            tg.append(sel[ok])
            sr.append(src[ok])
        tg = np.concatenate(tg)
        sr = np.concatenate(sr)
        order = np.lexsort((sr, tg))
        tg, sr = tg[order], sr[order]
        offs = np.zeros(len(keys) + 1, dtype=np.int64)
        np.add.at(offs, tg + 1, 1)
        return np.cumsum(offs), sr
