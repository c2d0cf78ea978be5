"""Dense, uncompressed kernel-independent FMM in float64 (Sections 2, 2.1.1,
2.2; M2L forms from Section 3.1 and Appendix A.1).

Test infrastructure only (see ``oracle/__init__``).

Passes, in the paper's order (Section 2, upward and downward pass):

* P2M (leaves): upward check potential phi_UC = K(UC, sources) q, then
  upward-equivalent densities q_UE = pinv(K(UC, UE)) phi_UC.
* M2M (levels d-1 .. 2): phi_UC(parent) = sum over existing children of
  K(UC_parent, UE_child) q_UE(child), then the same pseudo-inverse.
* Downward, levels 2 .. d: the check potential on the target's downward-check
  surface is the M2L sum over its interaction list, sum_sigma
  K(DC_tau, UE_sigma) q_UE(sigma) (the M2L matvec of Section 2.2; the
  source side is read as the upward-equivalent surface, where multipoles
  live), plus, from level 3 on, the L2L term K(DC_tau, DE_parent)
  q_DE(parent).  The two are summed first and the pseudo-inverse of
  K(DC, DE) is applied once.
* Leaves: L2P, phi(x) = K(x, DE_leaf) q_DE(leaf), plus P2P over the near
  field (Section 2, downward pass).

Every operator is built from box geometry at its own level (no homogeneity
scaling).  M2L matrices depend on the source/target centre offset only, so
one matrix per transfer vector and level is formed from that offset; the M2L
sum is accumulated per target in ascending transfer-vector index.

``m2l`` selects how each M2L matrix is applied: "dense" (the definition),
"fft" (the convolution of Appendix A.1, through ``fft_m2l``) or "blas" (the
compressed operator of Section 3.1, through ``blas_m2l``).

``check_order`` (P_c) sets the order of both check surfaces, ``order`` (P_e)
that of both equivalent surfaces.  The BLAS form may take P_c > P_e (more
check than equivalent points, often the more stable fit; Section 5.1, and
the P_e / P_c columns of the BLAS-M2L parameter table in Section 4), which
the convolution form cannot: its surfaces must be discretised alike.
Check-side arrays then have n_c = 6 (P_c - 1)^2 + 2 rows and
equivalent-side arrays n_e = 6 (P_e - 1)^2 + 2.
"""

from __future__ import annotations

import numpy as np

from . import blas_m2l, fft_m2l
from .kernel import kernel_matrix
from .linalg import pinv_apply, pinv_factors
from .surfaces import ALPHA_INNER, ALPHA_OUTER, n_surface, surface
from .tree import TRANSFER_VECTORS, Tree


def _octant_offset(o: int) -> np.ndarray:
    """Child-centre minus parent-centre in units of the child width."""
    return np.array([(o >> 0) & 1, (o >> 1) & 1, (o >> 2) & 1], dtype=np.float64) - 0.5


class KiFMM:
    """Plain FP64 kiFMM over a pruned uniform octree."""

    def __init__(self, sources, targets, depth: int, order: int,
                 origin=(0.0, 0.0, 0.0), width: float = 1.0, m2l: str = "dense",
                 svd_rel_tol: float = 0.0, svd_rel_tol_dir: float = -1.0,
                 alpha_inner: float = ALPHA_INNER, alpha_outer: float = ALPHA_OUTER,
                 check_order: int | None = None):
        if order < 2:
            raise ValueError("expansion order must be >= 2")
        self.tree = Tree(sources, targets, depth, origin, width)
        self.p = int(order)
        self.pc = self.p if check_order is None else int(check_order)
        if self.pc < self.p:
            raise ValueError("check order must be >= the expansion order")
        if m2l == "fft" and self.pc != self.p:
            raise ValueError("the convolution form needs equal check and equivalent orders")
        self.ns = n_surface(self.p)     # equivalent surfaces (n_e)
        self.nc = n_surface(self.pc)    # check surfaces (n_c)
        self.m2l = m2l
        self.tol = svd_rel_tol
        self.tol_dir = svd_rel_tol_dir
        self.ai = alpha_inner
        self.ao = alpha_outer
        self._comp = {}

    # ---- geometry ---------------------------------------------------------
    def w(self, level: int) -> float:
        return self.tree.width / 2 ** level

    def r(self, level: int) -> float:
        return 0.5 * self.w(level)

    def up_pinv(self, level: int):
        r = self.r(level)
        return pinv_factors(kernel_matrix(surface(self.pc, self.ao, r), surface(self.p, self.ai, r)))

    def down_pinv(self, level: int):
        r = self.r(level)
        return pinv_factors(kernel_matrix(surface(self.pc, self.ai, r), surface(self.p, self.ao, r)))

    def m2m_matrix(self, level: int, octant: int) -> np.ndarray:
        """K(UC of a parent at ``level``, UE of its child in ``octant``)."""
        rp, rc = self.r(level), self.r(level + 1)
        c = _octant_offset(octant) * self.w(level + 1)
        return kernel_matrix(surface(self.pc, self.ao, rp), surface(self.p, self.ai, rc, c))

    def l2l_matrix(self, level: int, octant: int) -> np.ndarray:
        """K(DC of a child at ``level`` in ``octant``, DE of its parent)."""
        rc, rp = self.r(level), self.r(level - 1)
        c = _octant_offset(octant) * self.w(level)
        return kernel_matrix(surface(self.pc, self.ai, rc, c), surface(self.p, self.ao, rp))

    def m2l_matrix(self, level: int, it: int) -> np.ndarray:
        """K(DC_tau, UE_sigma) for sigma = tau + t (anchors), t = TRANSFER_VECTORS[it]."""
        r = self.r(level)
        t = TRANSFER_VECTORS[it].astype(np.float64) * self.w(level)
        return kernel_matrix(surface(self.pc, self.ai, r), surface(self.p, self.ai, r, t))

    def compression(self, level: int) -> dict:
        if level not in self._comp:
            ks = blas_m2l.m2l_matrices(self.p, self.r(level), self.ai, check_order=self.pc)
            self._comp[level] = blas_m2l.compress(ks, self.tol, self.tol_dir)
        return self._comp[level]

    def m2l_apply(self, level: int, it: int, q: np.ndarray) -> np.ndarray:
        """Check potentials (m, n_c, nvec) of source densities q (m, n_e, nvec)."""
        if self.m2l == "dense":
            return np.einsum("ij,mjv->miv", self.m2l_matrix(level, it), q, optimize=True)
        if self.m2l == "blas":
            op = blas_m2l.applied_operator(self.compression(level), it)
            return np.einsum("ij,mjv->miv", op, q, optimize=True)
        if self.m2l == "fft":
            t = TRANSFER_VECTORS[it].astype(np.float64) * self.w(level)
            h = 2.0 * self.ai * self.r(level) / (self.p - 1)
            out = np.zeros_like(q)
            for m in range(q.shape[0]):
                for v in range(q.shape[2]):
                    out[m, :, v] = fft_m2l.check_potential(self.p, h, -t, q[m, :, v])
            return out
        raise ValueError(self.m2l)

    # ---- passes -----------------------------------------------------------
    def upward(self, charges: np.ndarray) -> list:
        """Upward-equivalent densities per level: arrays (n_boxes, n_s, nvec)."""
        tr = self.tree
        d = tr.depth
        q = np.atleast_2d(np.asarray(charges, dtype=np.float64))
        nvec = q.shape[0]
        qs = q[:, tr.src_perm]
        ys = tr.sources[tr.src_perm]
        leaves = tr.levels[d]
        centers = tr.center(d, np.arange(len(leaves)))
        phi = np.zeros((len(leaves), self.nc, nvec))
        for i in range(len(leaves)):
            s, e = tr.src_start[i], tr.src_end[i]
            if e > s:
                uc = surface(self.pc, self.ao, self.r(d), centers[i])
                phi[i] = kernel_matrix(uc, ys[s:e]) @ qs[:, s:e].T
        mult = [None] * (d + 1)
        mult[d] = self._apply_pinv(self.up_pinv(d), phi)
        for lev in range(d - 1, 1, -1):
            child_keys = tr.levels[lev + 1]
            parent = tr.index_of(lev, child_keys >> np.uint64(3))
            octant = (child_keys & np.uint64(7)).astype(np.int64)
            phi = np.zeros((len(tr.levels[lev]), self.nc, nvec))
            for o in range(8):
                sel = np.nonzero(octant == o)[0]
                if sel.size:
                    contrib = np.einsum("ij,mjv->miv", self.m2m_matrix(lev, o), mult[lev + 1][sel],
                                        optimize=True)
                    np.add.at(phi, parent[sel], contrib)
            mult[lev] = self._apply_pinv(self.up_pinv(lev), phi)
        return mult

    def _apply_pinv(self, factors, phi: np.ndarray) -> np.ndarray:
        """Equivalent densities (m, n_e, nvec) of check potentials (m, n_c, nvec)."""
        m, nc, nvec = phi.shape
        flat = phi.transpose(1, 0, 2).reshape(nc, m * nvec)
        out = pinv_apply(factors, flat)
        return out.reshape(out.shape[0], m, nvec).transpose(1, 0, 2).copy()

    def m2l_level(self, level: int, mult: np.ndarray, targets: np.ndarray | None = None) -> np.ndarray:
        """M2L check potentials at ``level`` for the boxes ``targets`` (all if None).

        ``mult`` holds the upward-equivalent densities of every box at the
        level; the result has shape (len(targets), n_c, nvec).
        """
        tr = self.tree
        offs, src, ti = tr.interactions(level)
        nb = len(tr.levels[level])
        tg = np.repeat(np.arange(nb), np.diff(offs))
        if targets is None:
            targets = np.arange(nb)
        pos = -np.ones(nb, dtype=np.int64)
        pos[targets] = np.arange(len(targets))
        keep = pos[tg] >= 0
        tg, src, ti = pos[tg[keep]], src[keep], ti[keep]
        out = np.zeros((len(targets), self.nc, mult.shape[2]))
        for it in range(len(TRANSFER_VECTORS)):
            sel = np.nonzero(ti == it)[0]
            if sel.size:
                out[tg[sel]] += self.m2l_apply(level, it, mult[src[sel]])
        return out

    def evaluate(self, charges: np.ndarray, sample: np.ndarray | None = None) -> np.ndarray:
        """Potentials (nvec, n_targets), or (nvec, len(sample)) at the target
        indices ``sample`` (original order)."""
        tr = self.tree
        d = tr.depth
        q = np.atleast_2d(np.asarray(charges, dtype=np.float64))
        nvec = q.shape[0]
        mult = self.upward(q)
        inv_perm = np.empty_like(tr.tgt_perm)
        inv_perm[tr.tgt_perm] = np.arange(len(tr.tgt_perm))
        if sample is None:
            sample = np.arange(tr.targets.shape[0])
        sample = np.asarray(sample, dtype=np.int64)
        sorted_pos = inv_perm[sample]
        tkeys = tr.tgt_keys_sorted[sorted_pos]
        need = [None] * (d + 1)
        need[d] = np.unique(tr.index_of(d, tkeys))
        for lev in range(d - 1, 1, -1):
            need[lev] = np.unique(tr.index_of(lev, tr.levels[lev + 1][need[lev + 1]] >> np.uint64(3)))
        local = [None] * (d + 1)
        for lev in range(2, d + 1):
            phi = self.m2l_level(lev, mult[lev], need[lev])
            if lev >= 3:
                keys = tr.levels[lev][need[lev]]
                par = tr.index_of(lev - 1, keys >> np.uint64(3))
                ppos = np.searchsorted(need[lev - 1], par)
                octant = (keys & np.uint64(7)).astype(np.int64)
                for o in range(8):
                    sel = np.nonzero(octant == o)[0]
                    if sel.size:
                        phi[sel] += np.einsum("ij,mjv->miv", self.l2l_matrix(lev, o),
                                              local[lev - 1][ppos[sel]], optimize=True)
            local[lev] = self._apply_pinv(self.down_pinv(lev), phi)
        # leaves: L2P + P2P at the requested targets
        noffs, nsrc = tr.near()
        ys = tr.sources[tr.src_perm]
        qs = q[:, tr.src_perm]
        xs = tr.targets[tr.tgt_perm]
        out = np.zeros((nvec, len(sample)))
        leaf_of = tr.index_of(d, tkeys)
        leaf_pos = np.searchsorted(need[d], leaf_of)
        centers = tr.center(d, need[d])
        for j, leaf in enumerate(need[d]):
            rows = np.nonzero(leaf_of == leaf)[0]
            x = xs[sorted_pos[rows]]
            de = surface(self.p, self.ao, self.r(d), centers[j])
            phi = kernel_matrix(x, de) @ local[d][leaf_pos[rows[0]]]
            nb = nsrc[noffs[leaf]:noffs[leaf + 1]]
            idx = np.concatenate([np.arange(tr.src_start[b], tr.src_end[b]) for b in nb])
            if idx.size:
                phi = phi + kernel_matrix(x, ys[idx]) @ qs[:, idx].T
            out[:, rows] = phi.T
        return out
