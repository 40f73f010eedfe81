"""The definition, densely (oracle; test infrastructure only).

Per energy E:
  z = E + i eta;  A = z I - H - Sigma_L(z) - Sigma_R(z)          (Eq. 1)
  G = A^-1 by LAPACK partial-pivot LU                              (Eq. 1)
  A_c,ii = sum_k |G_ik|^2 Gamma_c,k   (c = L, R)                   (Eq. 2 per contact)
  G^<_ii = i (f_L A_L,ii + f_R A_R,ii)                             (Eq. 2)
  T = sum_{i in L, j in R} Gamma_L,i |G_ij|^2 Gamma_R,j            (Caroli)
  A_eta,ii = 2 eta sum_k |G_ik|^2   (the broadening that eta itself adds)
Bond entries (bonds(): the desired off-diagonal entries, pairs (i, j) with H_ij != 0):
  G^r_ij from the same inverse; G^<_ij = i sum_c f_c (G_i,c V_c) . conj(G_j,c V_c)   (Eq. 2 entrywise)
with Gamma_c = V_c V_c^T (V_c = diag(sqrt(Gamma_c,k)) for per-site leads).
With dense=True each contact is a whole face with the dense self-energy block
of face.face_sigma (the DENSE case); then, with Gamma_c = V_c V_c^T,
  A_c,ii = || G_i,c V_c ||^2,    T = || V_L^T G_LR V_R ||_F^2  (= Tr Gamma_L G Gamma_R G^dagger)
With potential U (one value per site) the device Hamiltonian is H + diag(U): the on-site shift
of the self-consistent loop (scf.py).
Meant for n up to a few thousand sites.
"""
from __future__ import annotations

import numpy as np

from .negf import contact_sigmas, gamma_of, fermi
from .face import face_sigma


def system_matrix(dev, z, h=None, dense=False):
    """Dense A(z) = z I - H - Sigma_L - Sigma_R."""
    h = dev.dense_h() if h is None else h
    a = -h.astype(np.complex128, copy=True)
    a[np.diag_indices(dev.n)] += z
    if dense:
        for k, c in enumerate(dev.contacts):
            sites = np.asarray(c.sites, dtype=np.int64)
            a[np.ix_(sites, sites)] -= face_sigma(dev, k, z)[0]
        return a
    for sites, sig in contact_sigmas(dev, z):
        a[sites, sites] -= sig
    return a


def green(dev, energy: float, eta: float, h=None, dense=False):
    """Full G^r(E) as a dense matrix."""
    return np.linalg.inv(system_matrix(dev, energy + 1j * eta, h, dense))


def _h_of(dev, potential):
    h = dev.dense_h()
    if potential is not None:
        h[np.diag_indices(dev.n)] += np.asarray(potential, dtype=np.float64)
    return h


def solve(dev, energies, eta, kT, mu_L, mu_R, dense=False, potential=None):
    """Diagonals of G^r and G^<, spectral functions, transmission for each energy."""
    if dense:
        return _solve_dense(dev, energies, eta, kT, mu_L, mu_R, potential)
    energies = np.asarray(energies, dtype=np.float64)
    ne, n = len(energies), dev.n
    h = _h_of(dev, potential)
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


def _solve_dense(dev, energies, eta, kT, mu_L, mu_R, potential=None):
    energies = np.asarray(energies, dtype=np.float64)
    ne, n = len(energies), dev.n
    h = _h_of(dev, potential)
    out = {k: np.zeros((ne, n), np.complex128) for k in ("gr", "gl")}
    for k in ("a_l", "a_r", "a_eta"):
        out[k] = np.zeros((ne, n))
    out["trans"] = np.zeros(ne)
    fl = fermi(energies, mu_L, kT)
    fr = fermi(energies, mu_R, kT)
    ls = np.asarray(dev.contacts[0].sites, dtype=np.int64)
    rs = np.asarray(dev.contacts[1].sites, dtype=np.int64)
    for e, en in enumerate(energies):
        z = en + 1j * eta
        g = np.linalg.inv(system_matrix(dev, z, h, dense=True))
        v_l = face_sigma(dev, 0, z)[1]
        v_r = face_sigma(dev, 1, z)[1]
        a_l = (np.abs(g[:, ls] @ v_l) ** 2).sum(axis=1)
        a_r = (np.abs(g[:, rs] @ v_r) ** 2).sum(axis=1)
        out["gr"][e] = np.diag(g)
        out["a_l"][e] = a_l
        out["a_r"][e] = a_r
        out["a_eta"][e] = 2.0 * eta * (np.abs(g) ** 2).sum(axis=1)
        out["gl"][e] = 1j * (fl[e] * a_l + fr[e] * a_r)
        out["trans"][e] = (np.abs(v_l.T @ g[np.ix_(ls, rs)] @ v_r) ** 2).sum()
    return out


def bonds(dev, energies, eta, kT, mu_L, mu_R, pairs, dense=False):
    """G^r and G^< at the given (i, j) pairs for each energy (complex [n_e, n_pairs] each)."""
    energies = np.asarray(energies, dtype=np.float64)
    pairs = np.asarray(pairs, dtype=np.int64)
    h = dev.dense_h()
    fl = fermi(energies, mu_L, kT)
    fr = fermi(energies, mu_R, kT)
    out = {"gr": np.zeros((len(energies), len(pairs)), np.complex128),
           "gl": np.zeros((len(energies), len(pairs)), np.complex128)}
    i, j = pairs[:, 0], pairs[:, 1]
    for e, en in enumerate(energies):
        z = en + 1j * eta
        g = np.linalg.inv(system_matrix(dev, z, h, dense))
        out["gr"][e] = g[i, j]
        acc = np.zeros(len(pairs), np.complex128)
        for k, (c, f) in enumerate(zip(dev.contacts, (fl[e], fr[e]))):
            cs = np.asarray(c.sites, dtype=np.int64)
            if dense:
                v = face_sigma(dev, k, z)[1]
            else:
                v = np.diag(np.sqrt(gamma_of(contact_sigmas(dev, z)[k][1])))
            gv = g[:, cs] @ v
            acc += f * np.sum(gv[i] * np.conj(gv[j]), axis=1)
        out["gl"][e] = 1j * acc
    return out
