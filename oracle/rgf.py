"""Slab-wise recursive Green's function sweeps (oracle; test infrastructure only).

Section 2.1 of the paper: layers orthogonal to the transport axis make A block
tridiagonal; one sweep folds the layers on one side into the current layer,
the other sweep extracts the diagonal blocks.  Here the transport axis is the
contact axis x, layer n holds the sites with x-coordinate n, and the classic
left-/right-connected recurrences are used:

  gL_0 = A_00^-1,        gL_n = (A_nn - A_n,n-1 gL_n-1 A_n-1,n)^-1
  gR_N = A_NN^-1,        gR_n = (A_nn - A_n,n+1 gR_n+1 A_n+1,n)^-1
  G_NN = gL_N,           G_nn = gL_n + gL_n A_n,n+1 G_n+1,n+1 A_n+1,n gL_n
  G_n,N = -gL_n A_n,n+1 G_n+1,N           (column blocks to the right contact)
  G_0,0 = gR_0,          G_n,0 = -gR_n A_n,n-1 G_n-1,0   (to the left contact)

From the column blocks: A_L,ii = sum_{k in L} Gamma_L,k |G_ik|^2 (slab 0),
A_R,ii likewise with slab N, and T = sum_{k in L} Gamma_L,k A_R,kk.
Contacts must lie in the first (left) and last (right) layer.  With dense=True
the contacts are whole faces with the dense blocks of face.face_sigma
(Gamma_c = V_c V_c^T): A_c,ii = ||G_i,c V_c||^2 and T = ||V_L^T G_0N V_R||_F^2.
"""
from __future__ import annotations

import numpy as np

from .negf import contact_sigmas, gamma_of, fermi
from .face import face_sigma


def _layers(dev):
    x = dev.coords[:, 0]
    order = np.argsort(x, kind="stable")
    bounds = np.searchsorted(x[order], np.arange(x.max() + 2))
    return [order[bounds[k]:bounds[k + 1]] for k in range(x.max() + 1)]


def solve(dev, energies, eta, kT, mu_L, mu_R, dense=False):
    energies = np.asarray(energies, dtype=np.float64)
    ne, n = len(energies), dev.n
    layers = _layers(dev)
    nl = len(layers)
    h = dev.scipy_h().tocsr()
    hb = {}
    for a in range(nl):
        for b in (a - 1, a, a + 1):
            if 0 <= b < nl:
                hb[a, b] = h[layers[a]][:, layers[b]].toarray()
    pos = np.empty(n, dtype=np.int64)
    lay_of = np.empty(n, dtype=np.int64)
    for k, s in enumerate(layers):
        pos[s] = np.arange(len(s))
        lay_of[s] = k
    left, right = dev.contacts[0].sites, dev.contacts[1].sites
    assert np.all(lay_of[left] == 0) and np.all(lay_of[right] == nl - 1)
    out = {k: np.zeros((ne, n), np.complex128) for k in ("gr", "gl")}
    for k in ("a_l", "a_r"):
        out[k] = np.zeros((ne, n))
    out["trans"] = np.zeros(ne)
    fl = fermi(energies, mu_L, kT)
    fr = fermi(energies, mu_R, kT)
    for e, en in enumerate(energies):
        z = en + 1j * eta
        diag = []
        for k in range(nl):
            d = -hb[k, k].astype(np.complex128)
            d[np.diag_indices(len(layers[k]))] += z
            diag.append(d)
        if dense:
            ls, rs = np.asarray(left, dtype=np.int64), np.asarray(right, dtype=np.int64)
            (s_l, v_l), (s_r, v_r) = face_sigma(dev, 0, z), face_sigma(dev, 1, z)
            diag[0][np.ix_(pos[ls], pos[ls])] -= s_l
            diag[nl - 1][np.ix_(pos[rs], pos[rs])] -= s_r
        else:
            (ls, sl), (rs, sr) = contact_sigmas(dev, z)
            diag[0][pos[ls], pos[ls]] -= sl
            diag[nl - 1][pos[rs], pos[rs]] -= sr
        off = {key: -v for key, v in hb.items() if key[0] != key[1]}   # A_ab = -H_ab
        gl = [None] * nl
        gl[0] = np.linalg.inv(diag[0])
        for k in range(1, nl):
            gl[k] = np.linalg.inv(diag[k] - off[k, k - 1] @ gl[k - 1] @ off[k - 1, k])
        gr = [None] * nl
        gr[nl - 1] = np.linalg.inv(diag[nl - 1])
        for k in range(nl - 2, -1, -1):
            gr[k] = np.linalg.inv(diag[k] - off[k, k + 1] @ gr[k + 1] @ off[k + 1, k])
        gdiag = [None] * nl
        gdiag[nl - 1] = gl[nl - 1]
        for k in range(nl - 2, -1, -1):
            gdiag[k] = gl[k] + gl[k] @ off[k, k + 1] @ gdiag[k + 1] @ off[k + 1, k] @ gl[k]
        col_r = [None] * nl       # G_{k, N}
        col_r[nl - 1] = gdiag[nl - 1]
        for k in range(nl - 2, -1, -1):
            col_r[k] = -gl[k] @ off[k, k + 1] @ col_r[k + 1]
        col_l = [None] * nl       # G_{k, 0}
        col_l[0] = gr[0]
        for k in range(1, nl):
            col_l[k] = -gr[k] @ off[k, k - 1] @ col_l[k - 1]
        if dense:
            for k in range(nl):
                s = layers[k]
                out["gr"][e, s] = np.diag(gdiag[k])
                out["a_l"][e, s] = (np.abs(col_l[k][:, pos[ls]] @ v_l) ** 2).sum(axis=1)
                out["a_r"][e, s] = (np.abs(col_r[k][:, pos[rs]] @ v_r) ** 2).sum(axis=1)
            g_lr = col_r[0][np.ix_(pos[ls], pos[rs])]
            out["trans"][e] = (np.abs(v_l.T @ g_lr @ v_r) ** 2).sum()
            out["gl"][e] = 1j * (fl[e] * out["a_l"][e] + fr[e] * out["a_r"][e])
            continue
        gam_l, gam_r = gamma_of(sl), gamma_of(sr)
        for k in range(nl):
            s = layers[k]
            out["gr"][e, s] = np.diag(gdiag[k])
            out["a_l"][e, s] = (np.abs(col_l[k][:, pos[ls]]) ** 2) @ gam_l
            out["a_r"][e, s] = (np.abs(col_r[k][:, pos[rs]]) ** 2) @ gam_r
        out["trans"][e] = gam_l @ out["a_r"][e, ls]
        out["gl"][e] = 1j * (fl[e] * out["a_l"][e] + fr[e] * out["a_r"][e])
    return out
