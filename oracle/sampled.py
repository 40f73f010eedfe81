"""Sampled rows of G^r by sparse LU (oracle; test infrastructure only).

For any device size: factor A(E) = z I - H - Sigma with a general sparse LU
(SuperLU, partial pivoting) and solve A^T x = e_s, so that x_k = (A^-1)_{s,k}
is row s of G^r.  From that row (Eq. 1 and Eq. 2 for diagonal Sigma^<):

  G^r_ss = x_s,   A_c,ss = sum_{k in c} Gamma_c,k |x_k|^2,
  G^<_ss = i (f_L A_L,ss + f_R A_R,ss).

The transmission T = sum_{i in L} Gamma_L,i A_R,ii needs the rows of every
left-contact site; it is computed only when asked for.

Each solve is refined twice (iterative refinement): the residual e_s - A^T x
is accumulated in extended precision (numpy longdouble) and the correction is
solved with the same factors, so the rows are accurate to working precision
rather than to eps * cond(A).

Rows and columns are first permuted by a geometric nested-dissection order
(bisect the longest box axis, separator last) only to keep the sparse
factors small; a symmetric permutation does not change A^-1, and SuperLU's
partial row pivoting keeps the factorisation stable in any column order.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from .negf import contact_sigmas, gamma_of, fermi


def _bisection_order(coords, leaf=4):
    """Sites ordered as: first half, second half, separator plane (recursively)."""
    out = []

    def rec(idx):
        c = coords[idx]
        lo, hi = c.min(0), c.max(0)
        ext = hi - lo + 1
        a = int(np.argmax(ext))
        if ext[a] <= leaf or ext[a] < 3:
            out.append(idx)
            return
        cut = lo[a] + ext[a] // 2
        rec(idx[c[:, a] < cut])
        rec(idx[c[:, a] > cut])
        out.append(idx[c[:, a] == cut])

    rec(np.arange(len(coords)))
    return np.concatenate(out)


class _Factor:
    """LU of P A P^T; solves are returned in the original site order."""

    def __init__(self, dev, z, refine=2):
        h = dev.scipy_h()
        a = (-h).tolil()
        a.setdiag(a.diagonal() + z)
        for sites, sig in contact_sigmas(dev, z):
            for s, v in zip(sites, sig):
                a[s, s] -= v
        a = sp.csc_matrix(a)
        self.p = _bisection_order(np.asarray(dev.coords))
        self.lu = spl.splu(a[self.p][:, self.p].tocsc(), permc_spec="NATURAL")
        at = a.T.tocsr()                     # rows of A^T, for the residual
        self.at_ptr = at.indptr
        self.at_col = at.indices
        self.at_val = at.data.astype(np.clongdouble)
        self.refine = refine

    def _solve_t0(self, b):
        x = np.empty_like(b)
        x[self.p] = self.lu.solve(b[self.p], trans="T")
        return x

    def _residual(self, b, x):
        """b - A^T x, accumulated in extended precision."""
        prod = self.at_val[:, None] * x[self.at_col]
        # every row holds its diagonal entry, so no row segment is empty
        ax = np.add.reduceat(prod, self.at_ptr[:-1], axis=0)
        return b.astype(np.clongdouble) - ax

    def solve_t(self, b):
        """x = A^-T b, with iterative refinement."""
        x = self._solve_t0(b).astype(np.clongdouble)
        for _ in range(self.refine):
            r = self._residual(b, x)
            x = x + self._solve_t0(r.astype(np.complex128))
        return x.astype(np.complex128)


def _factor(dev, z):
    return _Factor(dev, z)


def _rows(lu, n, sites):
    b = np.zeros((n, len(sites)), dtype=np.complex128)
    b[np.asarray(sites), np.arange(len(sites))] = 1.0
    return lu.solve_t(b)                  # column j = row sites[j] of A^-1


def solve_sites(dev, energies, eta, kT, mu_L, mu_R, sites, want_trans=False, chunk=128):
    energies = np.asarray(energies, dtype=np.float64)
    sites = np.asarray(sites, dtype=np.int64)
    ne = len(energies)
    out = {k: np.zeros((ne, len(sites)), np.complex128) for k in ("gr", "gl")}
    for k in ("a_l", "a_r"):
        out[k] = np.zeros((ne, len(sites)))
    out["trans"] = np.full(ne, np.nan)
    fl = fermi(energies, mu_L, kT)
    fr = fermi(energies, mu_R, kT)
    for e, en in enumerate(energies):
        z = en + 1j * eta
        lu = _factor(dev, z)
        (ls, sl), (rs, sr) = contact_sigmas(dev, z)
        gam_l, gam_r = gamma_of(sl), gamma_of(sr)
        for c0 in range(0, len(sites), chunk):
            blk = sites[c0:c0 + chunk]
            x = _rows(lu, dev.n, blk)
            out["gr"][e, c0:c0 + len(blk)] = x[blk, np.arange(len(blk))]
            out["a_l"][e, c0:c0 + len(blk)] = gam_l @ (np.abs(x[ls]) ** 2)
            out["a_r"][e, c0:c0 + len(blk)] = gam_r @ (np.abs(x[rs]) ** 2)
        out["gl"][e] = 1j * (fl[e] * out["a_l"][e] + fr[e] * out["a_r"][e])
        if want_trans:
            t = 0.0
            for c0 in range(0, len(ls), chunk):
                blk = ls[c0:c0 + chunk]
                x = _rows(lu, dev.n, blk)
                t += gam_l[c0:c0 + len(blk)] @ (gam_r @ (np.abs(x[rs]) ** 2))
            out["trans"][e] = t
    return out
