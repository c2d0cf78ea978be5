"""Backward-stable pseudo-inverse (Section 2.1.1).

Test infrastructure only (see ``oracle/__init__``).

q = V_eps (Sigma_eps^{-1} U_eps^T) Phi, stored as two factors.  Singular
values at or below eps = (alpha + rho) sigma_0 are dropped, with absolute
tolerance alpha = 0 and relative tolerance rho = max(M, N) * machine epsilon
of float64, which is SciPy's default rule.
"""

from __future__ import annotations

import numpy as np


def pinv_factors(k: np.ndarray):
    """Return (V, Ut) with pinv(k) = V @ Ut, Ut = Sigma^{-1} U^T (kept part)."""
    u, s, vt = np.linalg.svd(k, full_matrices=False)
    tol = max(k.shape) * np.finfo(np.float64).eps * s[0]
    keep = s > tol
    v = vt[keep].T
    ut = (u[:, keep] / s[keep]).T
    return v, ut


def pinv_apply(factors, phi: np.ndarray) -> np.ndarray:
    """Apply the two-factor pseudo-inverse: V @ (Ut @ phi)."""
    v, ut = factors
    return v @ (ut @ phi)
