"""Equivalent and check surfaces of the kiFMM (Section 2.1.1; the point count
6 (P-1)^2 + 2 is stated in Appendix A.3).

Test infrastructure only (see ``oracle/__init__``).

A surface of order p around a box with centre c and half-width r is the set
of points c + alpha r (-1 + 2 i / (p-1)) for integer i in [0, p-1]^3 on the
boundary of that lattice (min(i) = 0 or max(i) = p-1), listed with i_x
slowest and i_z fastest.  The radii are not fixed by the paper; the values
used are alpha = 1.05 for the upward-equivalent and downward-check surfaces
and alpha = 2.95 for the upward-check and downward-equivalent surfaces
(parity unpinned convention, shared with the library's header).  The paper
requires the upward-equivalent and downward-check surfaces to coincide
relative to their box for the convolution form of M2L (Section 2.2).
"""

from __future__ import annotations

import itertools

import numpy as np

ALPHA_INNER = 1.05
ALPHA_OUTER = 2.95


def n_surface(p: int) -> int:
    return 6 * (p - 1) ** 2 + 2


def lattice_indices(p: int) -> np.ndarray:
    """Integer lattice positions (n_s, 3) of the surface points."""
    idx = [i for i in itertools.product(range(p), repeat=3) if min(i) == 0 or max(i) == p - 1]
    return np.array(idx, dtype=np.int64)


def surface(p: int, alpha: float, half_width: float, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Surface points (n_s, 3) for a box of the given half-width and centre."""
    i = lattice_indices(p).astype(np.float64)
    return np.asarray(center, dtype=np.float64) + alpha * half_width * (-1.0 + 2.0 * i / (p - 1))
