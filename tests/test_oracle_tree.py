"""Pins of the oracle's octree, keys and lists (Section 2; Section 3.1 for the
189 / 316 counts) against brute force from the definitions."""
import itertools
import json
import os

import numpy as np
import pytest

import workloads
from oracle import tree as T


def counts(repo_root):
    with open(os.path.join(repo_root, "tests", "golden", "paper_counts.json")) as f:
        return json.load(f)


def direct_anchor(points, level):
    # anchors from the subdivision itself, level by level, without keys
    u = points.copy()
    a = np.zeros(points.shape, dtype=np.int64)
    lo = np.zeros(points.shape)
    size = 1.0
    for _ in range(level):
        size /= 2
        bit = (u >= lo + size).astype(np.int64)
        a = 2 * a + bit
        lo = lo + bit * size
    return a


def test_anchor_matches_recursive_subdivision():
    pts = workloads.uniform_cube(5000, 11)
    for lev in (1, 3, 5):
        assert np.array_equal(T.leaf_anchors(pts, (0, 0, 0), 1.0, lev), direct_anchor(pts, lev))


def test_keys_roundtrip_parent_and_zorder():
    rng = np.random.default_rng(5)
    for lev in (1, 2, 4, 7):
        a = rng.integers(0, 2 ** lev, size=(500, 3))
        k = T.morton_keys(a, lev)
        assert np.array_equal(T.key_anchors(k, lev), a)
        assert np.array_equal(k >> np.uint64(3), T.morton_keys(a >> 1, lev - 1))
        # octant of the child: x is bit 0, y bit 1, z bit 2
        o = (k & np.uint64(7)).astype(np.int64)
        assert np.array_equal(o, (a[:, 0] & 1) + 2 * (a[:, 1] & 1) + 4 * (a[:, 2] & 1))
        # key order = order of the octant path from the root (Z-order)
        path = [tuple(((a[i] >> (lev - 1 - b)) & 1) @ np.array([1, 2, 4]) for b in range(lev))
                for i in range(len(a))]
        order_keys = np.argsort(k, kind="stable")
        order_path = sorted(range(len(a)), key=lambda i: path[i])
        assert [path[i] for i in order_keys] == [path[i] for i in order_path]


def test_boundary_point_and_outside_rejected():
    a = T.leaf_anchors(np.array([[1.0, 0.0, 0.5]]), (0, 0, 0), 1.0, 3)
    assert a.tolist() == [[7, 0, 4]]
    with pytest.raises(ValueError):
        T.leaf_anchors(np.array([[1.0000001, 0.5, 0.5]]), (0, 0, 0), 1.0, 3)


def brute_lists(tr, level):
    keys = tr.levels[level]
    a = T.key_anchors(keys, level)
    out = []
    for i in range(len(keys)):
        lst = []
        for j in range(len(keys)):
            near = np.max(np.abs(a[i] - a[j])) <= 1
            pnear = np.max(np.abs(a[i] // 2 - a[j] // 2)) <= 1
            if pnear and not near:
                t = tuple(a[j] - a[i])
                lst.append((int(keys[j]), j, T.TRANSFER_VECTORS.tolist().index(list(t))))
        lst.sort()
        out.append(lst)
    return out


@pytest.mark.parametrize("kind", ["uniform", "sphere"])
def test_interaction_lists_match_brute_force(kind):
    if kind == "uniform":
        pts = workloads.uniform_cube(3000, 12)
        tr = T.Tree(pts, pts, 3)
    else:
        pts = workloads.sphere_surface(3000, 13)
        tr = T.Tree(pts, pts, 4, (-1, -1, -1), 2.0)
    for lev in range(2, tr.depth + 1):
        offs, src, ti = tr.interactions(lev)
        brute = brute_lists(tr, lev)
        for i, lst in enumerate(brute):
            got = list(zip(src[offs[i]:offs[i + 1]].tolist(), ti[offs[i]:offs[i + 1]].tolist()))
            assert got == [(j, t) for _, j, t in lst]


def test_near_lists_match_brute_force():
    pts = workloads.sphere_surface(2000, 14)
    tr = T.Tree(pts, pts, 3, (-1, -1, -1), 2.0)
    offs, src = tr.near()
    a = T.key_anchors(tr.levels[3], 3)
    for i in range(len(a)):
        want = [j for j in range(len(a)) if np.max(np.abs(a[i] - a[j])) <= 1]
        assert src[offs[i]:offs[i + 1]].tolist() == want


def test_counts_on_full_levels(repo_root):
    g = counts(repo_root)
    assert len(T.TRANSFER_VECTORS) == g["transfer_vectors_max"]["value"]
    # every box of a full level 4 tree; pair count (6n-8)^3 - (3n-2)^3
    n = 16
    a = np.array(list(itertools.product(range(n), repeat=3)))
    pts = (a + 0.5) / n
    tr = T.Tree(pts, pts, 4)
    for lev in (2, 3, 4):
        offs, src, ti = tr.interactions(lev)
        m = 2 ** lev
        assert offs[-1] == (6 * m - 8) ** 3 - (3 * m - 2) ** 3
        assert np.max(np.diff(offs)) <= g["interaction_list_max"]["value"]
        assert len(np.unique(ti)) == 316
    # an interior box: 189 sources
    anc = T.key_anchors(tr.levels[4], 4)
    i = int(np.nonzero((anc == [8, 8, 8]).all(axis=1))[0][0])
    assert offs[i + 1] - offs[i] == 189


def test_point_order_is_key_then_index():
    pts = workloads.uniform_cube(4000, 15)
    pts[10] = pts[20]
    tr = T.Tree(pts, pts, 4)
    k = tr.src_keys_sorted
    assert np.all(k[:-1] <= k[1:])
    same = k[:-1] == k[1:]
    assert np.all(tr.src_perm[:-1][same] < tr.src_perm[1:][same])
