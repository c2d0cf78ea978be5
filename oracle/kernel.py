"""Laplace kernel and direct summation (Section 1: the N-body sum and the 3D
Laplace kernel K(x, y) = 1 / (4 pi |x - y|)).

Test infrastructure only (see ``oracle/__init__``).

Self interaction: the paper takes sources equal to targets (Section 4) and is
silent on r = 0; here K(x, y) = 0 when x and y are bitwise equal.
"""

from __future__ import annotations

import numpy as np

INV_4PI = 1.0 / (4.0 * np.pi)


def kernel_matrix(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Dense [K(x_i, y_j)] for x (m, 3) and y (n, 3), float64."""
    d = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    with np.errstate(divide="ignore"):
        k = INV_4PI / r
    k[r == 0.0] = 0.0
    return k


def direct(sources: np.ndarray, charges: np.ndarray, targets: np.ndarray,
           chunk: int = 2048) -> np.ndarray:
    """phi_i = sum_j K(x_i, y_j) q_j for every charge vector.

    ``charges`` has shape (nvec, n_src); the result has shape (nvec, n_tgt).
    """
    q = np.atleast_2d(charges)
    out = np.zeros((q.shape[0], targets.shape[0]))
    for s in range(0, targets.shape[0], chunk):
        k = kernel_matrix(targets[s:s + chunk], sources)
        out[:, s:s + chunk] = (k @ q.T).T
    return out


def rel_l2(approx: np.ndarray, exact: np.ndarray) -> float:
    """Relative L2 error over all entries (Section 4, the L2 error metric)."""
    a = np.asarray(approx, dtype=np.float64).ravel()
    e = np.asarray(exact, dtype=np.float64).ravel()
    den = np.sqrt(np.sum(e * e))
    return float(np.sqrt(np.sum((a - e) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(a * a)))
