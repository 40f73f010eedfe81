"""The definition, densely (oracle; test infrastructure only).

Per energy E:
  z = E + i eta;  A = z I - H - Sigma_L(z) - Sigma_R(z)          (Eq. 1)
  G = A^-1 by LAPACK partial-pivot LU                              (Eq. 1)
  A_c,ii = sum_k |G_ik|^2 Gamma_c,k   (c = L, R)                   (Eq. 2 per contact)
  G^<_ii = i (f_L A_L,ii + f_R A_R,ii)                             (Eq. 2)
  T = sum_{i in L, j in R} Gamma_L,i |G_ij|^2 Gamma_R,j            (Caroli)
  A_eta,ii = 2 eta sum_k |G_ik|^2   (the broadening that eta itself adds)
Meant for n up to a few thousand sites.
"""
from __future__ import annotations

import numpy as np

from .negf import contact_sigmas, gamma_of, fermi


def system_matrix(dev, z, h=None):
    """Dense A(z) = z I - H - Sigma_L - Sigma_R."""
    h = dev.dense_h() if h is None else h
    a = -h.astype(np.complex128, copy=True)
    a[np.diag_indices(dev.n)] += z
    for sites, sig in contact_sigmas(dev, z):
        a[sites, sites] -= sig
    return a


def green(dev, energy: float, eta: float, h=None):
    """Full G^r(E) as a dense matrix."""
    return np.linalg.inv(system_matrix(dev, energy + 1j * eta, h))


def solve(dev, energies, eta, kT, mu_L, mu_R):
    """Diagonals of G^r and G^<, spectral functions, transmission for each energy."""
    energies = np.asarray(energies, dtype=np.float64)
    ne, n = len(energies), dev.n
    h = dev.dense_h()
    out = {k: np.zeros((ne, n), np.complex128) for k in ("gr", "gl")}
    for k in ("a_l", "a_r", "a_eta"):
        out[k] = np.zeros((ne, n))
    out["trans"] = np.zeros(ne)
    fl = fermi(energies, mu_L, kT)
    fr = fermi(energies, mu_R, kT)
    for e, en in enumerate(energies):
        z = en + 1j * eta
        g = np.linalg.inv(system_matrix(dev, z, h))
        (ls, sl), (rs, sr) = contact_sigmas(dev, z)
        gam_l, gam_r = gamma_of(sl), gamma_of(sr)
        mag = np.abs(g) ** 2
        a_l = mag[:, ls] @ gam_l
        a_r = mag[:, rs] @ gam_r
        out["gr"][e] = np.diag(g)
        out["a_l"][e] = a_l
        out["a_r"][e] = a_r
        out["a_eta"][e] = 2.0 * eta * mag.sum(axis=1)
        out["gl"][e] = 1j * (fl[e] * a_l + fr[e] * a_r)
        out["trans"][e] = gam_l @ mag[np.ix_(ls, rs)] @ gam_r
    return out
