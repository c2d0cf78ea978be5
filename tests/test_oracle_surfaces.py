"""Pins of the equivalent/check surfaces (Section 2.1.1; point count from
Appendix A.3)."""
import json
import os

import numpy as np
import pytest

from oracle import surfaces


def golden(repo_root):
    with open(os.path.join(repo_root, "tests", "golden", "paper_counts.json")) as f:
        return json.load(f)


def test_counts_match_paper(repo_root):
    g = golden(repo_root)["surface_points"]
    for p, n in g.items():
        if p.startswith("_"):
            continue
        assert surfaces.n_surface(int(p)) == n
        assert len(surfaces.lattice_indices(int(p))) == n


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 8, 10])
def test_points_on_cube_surface(p):
    pts = surfaces.surface(p, 2.95, 0.25, center=(0.1, -0.2, 0.3))
    d = np.abs(pts - np.array([0.1, -0.2, 0.3]))
    assert np.allclose(np.max(d, axis=1), 2.95 * 0.25, rtol=1e-14)
    # distinct points, and every lattice boundary point is present
    assert len(np.unique(np.round(pts, 12), axis=0)) == surfaces.n_surface(p)
    idx = surfaces.lattice_indices(p)
    brute = sum(1 for i in range(p) for j in range(p) for k in range(p)
                if 0 in (i, j, k) or p - 1 in (i, j, k))
    assert len(idx) == brute
