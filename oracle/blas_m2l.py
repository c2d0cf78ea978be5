"""SVD-compressed M2L operators (Section 3.1).

Test infrastructure only (see ``oracle/__init__``).

For one level, the 316 M2L matrices K_t (rows: the target's downward check
surface, columns: the source's upward equivalent surface) are stacked into
K_fat = [K_1 ... K_T] and K_thin = [K_1; ...; K_T].  Their SVDs give U (left
vectors of K_fat) and S (right vectors of K_thin); with the first k columns
kept, K_t ~ U C_t S^T with C_t = U^T K_t S.  Directional recompression keeps
the first k_t singular triplets of each C_t: C_t ~ Ubar_t Vbar'_t^T with
Vbar'_t = Vbar_t Sigmabar_t.

Threshold reading (the paper's "singular value threshold" is not defined
further): k = #{sigma_i(K_fat) > tol * sigma_0(K_fat)}, capped at n_e (the
right vectors K_thin has) when check surfaces are finer than equivalent ones,
since C_t is k x k for one k, and k_t =
#{sigma_i(C_t) > tol_dir * sigma_0(C_t)}; tol = 0 keeps full rank and
tol_dir < 0 skips recompression.  The operator the method applies,
U Ubar_t Vbar'_t^T S^T, does not depend on the signs or bases the SVD routine
returns when the kept singular values are separated from the dropped ones,
so it is the quantity compared with the library.
"""

from __future__ import annotations

import numpy as np

from .kernel import kernel_matrix
from .surfaces import ALPHA_INNER, surface
from .tree import TRANSFER_VECTORS


def m2l_matrices(p: int, half_width: float, alpha: float = ALPHA_INNER,
                 check_order: int | None = None) -> list[np.ndarray]:
    """K_t for the 316 transfer vectors at a level with box half-width r:
    target check surface (order check_order, default p) around 0, source
    equivalent surface (order p) around t * 2r; n_c x n_e each."""
    x = surface(p if check_order is None else check_order, alpha, half_width)
    out = []
    for t in TRANSFER_VECTORS:
        y = surface(p, alpha, half_width, center=t * 2.0 * half_width)
        out.append(kernel_matrix(x, y))
    return out


def _rank(s: np.ndarray, tol: float) -> int:
    if tol <= 0.0:
        return int(np.sum(s > 0.0))
    return int(np.sum(s > tol * s[0]))


def compress(ks: list[np.ndarray], tol: float, tol_dir: float) -> dict:
    """Fat/thin SVD compression plus directional recompression."""
    kfat = np.hstack(ks)
    kthin = np.vstack(ks)
    u, sfat, _ = np.linalg.svd(kfat, full_matrices=False)
    _, sthin, st = np.linalg.svd(kthin, full_matrices=False)
    # one rank k for both sides (C_t is k x k), at most the number of right
    # vectors K_thin has (n_e, below n_c when the check order is the higher)
    k = min(_rank(sfat, tol), st.shape[0])
    uk = u[:, :k]
    sk = st[:k].T
    ubar, vbarp, kts = [], [], []
    for kt_mat in ks:
        c = uk.T @ kt_mat @ sk
        if tol_dir < 0.0:
            ubar.append(np.eye(k))
            vbarp.append(c.T.copy())
            kts.append(k)
            continue
        cu, cs, cvt = np.linalg.svd(c)
        r = _rank(cs, tol_dir)
        ubar.append(cu[:, :r])
        vbarp.append(cvt[:r].T * cs[:r])
        kts.append(r)
    return dict(U=uk, S=sk, k=k, sigma_fat=sfat, sigma_thin=sthin,
                Ubar=ubar, Vbarp=vbarp, kt=np.array(kts))


def applied_operator(comp: dict, it: int) -> np.ndarray:
    """Dense n_c x n_e operator U Ubar_t Vbar'_t^T S^T for transfer index it."""
    return comp["U"] @ comp["Ubar"][it] @ comp["Vbarp"][it].T @ comp["S"].T
