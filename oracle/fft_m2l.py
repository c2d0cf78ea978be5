"""Reference FFT-M2L of one source/target box pair (Appendix A.1).

Test infrastructure only (see ``oracle/__init__``); used to pin that the
convolution form reproduces the dense M2L exactly (Section 5.1 calls the
FFT form exact for translation-invariant kernels).

Reading of Appendix A.1 (the printed 1D index expression is off by one and is
not followed): the surface lattice of P points per axis is embedded in a
convolution grid of 2P points per axis.  With h the lattice spacing,
target check point a and source equivalent point b (integer lattice
positions in [0, P-1]^3) interact through K(c_tau - c_sigma + h (a - b)),
which depends on a - b only.  The kernel sequence G[m] = K(c_tau - c_sigma +
h m) for m in [-(P-1), P-1]^3 is stored at grid index m mod 2P (the index P
in any axis is zero padding); the densities are placed at their lattice
positions with zeros elsewhere.  The check potential at lattice point a is
entry a of the inverse DFT of DFT(G) * DFT(D).  Since 2P > 2P - 1 the
circular convolution does not wrap onto used entries.  The kernel being real,
only (2P)^2 (P + 1) Fourier coefficients are independent (Appendix A.2).

The same argument holds for any grid of n >= 2P - 1 points per axis (the
offsets m span 2P - 1 values); every function takes the grid size ``n``,
2P by default as in the paper.
"""

from __future__ import annotations

import numpy as np

from .kernel import INV_4PI
from .surfaces import lattice_indices


def kernel_grid(p: int, spacing: float, dc: np.ndarray, n: int | None = None) -> np.ndarray:
    """G on the n^3 grid (n = 2p by default) for centre offset dc = c_target - c_source."""
    n = 2 * p if n is None else n
    if n < 2 * p - 1:
        raise ValueError("grid too small: the circular convolution would wrap")
    g = np.zeros((n, n, n))
    r = np.arange(-(p - 1), p)
    mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
    d = np.stack([dc[0] + spacing * mx, dc[1] + spacing * my, dc[2] + spacing * mz], axis=-1)
    val = INV_4PI / np.sqrt(np.sum(d * d, axis=-1))
    g[mx % n, my % n, mz % n] = val
    return g


def density_grid(p: int, q: np.ndarray, n: int | None = None) -> np.ndarray:
    """Densities (n_s,) on their lattice positions of the n^3 grid."""
    n = 2 * p if n is None else n
    d = np.zeros((n, n, n))
    idx = lattice_indices(p)
    d[idx[:, 0], idx[:, 1], idx[:, 2]] = q
    return d


def kernel_spectrum(p: int, spacing: float, dc: np.ndarray, n: int | None = None) -> np.ndarray:
    """Real-to-complex spectrum, shape (n, n, n // 2 + 1)."""
    return np.fft.rfftn(kernel_grid(p, spacing, dc, n))


def check_potential(p: int, spacing: float, dc: np.ndarray, q: np.ndarray,
                    n: int | None = None) -> np.ndarray:
    """Check potential (n_s,) of densities q through the convolution grid."""
    n = 2 * p if n is None else n
    spec = kernel_spectrum(p, spacing, dc, n) * np.fft.rfftn(density_grid(p, q, n))
    full = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
    idx = lattice_indices(p)
    return full[idx[:, 0], idx[:, 1], idx[:, 2]]


def storage_words(p: int) -> int:
    """Complex words of kernel spectra for 26 source clusters x 64 box pairs
    in the sibling-cluster layout (Appendix A.1-A.2), per level."""
    return 26 * 64 * (2 * p) ** 2 * (p + 1)
