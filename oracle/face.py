"""DENSE contact self-energy of a whole face (oracle; test infrastructure only).

The paper's DENSE case (cuboid experiments with dense self-energy matrices,
Section 3.1.2; the open-boundary caveat of Section 2.3): the contact is a whole
face of the device, and its lead is the semi-infinite continuation of that
face.  Layer m of the lead is a copy of the face lattice: on-site ``eps0``,
hopping ``t_l`` between nearest neighbours inside the layer and between a site
and its copy in the next layer.  Each face site couples to its copy in the
first lead layer with hopping ``t_c``.  So, with H00 = eps0 I + t_l Adj (Adj the
face's nearest-neighbour adjacency) and H01 = t_l I,

  g_s = (z - H00 - H01 g_s H01^T)^-1      (surface Green's function of the lead)
  Sigma = t_c^2 g_s,   Gamma = i (Sigma - Sigma^dagger)

Sigma is a dense complex-symmetric |face| x |face| block.

Evaluation: Adj = U diag(mu) U^T (numpy.linalg.eigh; U real orthogonal).  In
that basis H00 and H01 are both diagonal, so every transverse mode m is a 1D
chain (on-site eps0 + t_l mu_m, hopping t_l) whose surface function is the
decaying root of t_l^2 g^2 - (z - eps0 - t_l mu_m) g + 1 = 0 (negf.sigma_lead
with unit coupling).  Sigma = t_c^2 U diag(g_m) U^T and Gamma = V V^T with
V = U diag(sqrt(gamma_m)), gamma_m = -2 t_c^2 Im g_m >= 0.

Pins (tests): the surface Dyson equation above, Sancho-Rubio decimation
(`decimation`, an independent iteration), the one-site face (the 1D chain),
and the clean wire whose transmission counts the open transverse modes.

The face's two transverse axes are the ones along which its sites vary; the
normal axis is the one along which both contacts are flat and differ.
"""
from __future__ import annotations

import numpy as np

from .negf import sigma_lead


def normal_axis(dev) -> int:
    """Axis along which each contact is flat and the two contacts differ."""
    c0 = dev.coords[np.asarray(dev.contacts[0].sites)]
    c1 = dev.coords[np.asarray(dev.contacts[1].sites)]
    for a in range(3):
        if np.all(c0[:, a] == c0[0, a]) and np.all(c1[:, a] == c1[0, a]) and c0[0, a] != c1[0, a]:
            return a
    raise ValueError("the contacts are not two parallel faces")


def face_adjacency(dev, k: int) -> np.ndarray:
    """Nearest-neighbour adjacency (0/1) of contact k's sites within its face, in contact order."""
    ax = normal_axis(dev)
    tr = [a for a in range(3) if a != ax]
    xy = dev.coords[np.asarray(dev.contacts[k].sites)][:, tr].astype(np.int64)
    d = np.abs(xy[:, None, :] - xy[None, :, :]).sum(axis=2)
    return (d == 1).astype(np.float64)


def face_modes(dev, k: int):
    """(U, mu): transverse eigenvectors (columns) and eigenvalues of the face adjacency."""
    mu, u = np.linalg.eigh(face_adjacency(dev, k))
    return u, mu


def face_sigma(dev, k: int, z):
    """(Sigma, V) of contact k at complex energy z: Sigma dense, Gamma = V V^T."""
    c = dev.contacts[k]
    u, mu = face_modes(dev, k)
    g = np.array([complex(sigma_lead(z, c.lead_onsite + c.lead_hopping * m, c.lead_hopping, 1.0)) for m in mu])
    sig = (c.coupling ** 2) * (u * g) @ u.T
    gam = np.maximum(-2.0 * (c.coupling ** 2) * g.imag, 0.0)
    return sig, u * np.sqrt(gam)


def decimation(dev, k: int, z, tol: float = 1e-15, max_iter: int = 200):
    """Sigma of contact k by Sancho-Rubio decimation (Lopez Sancho, Lopez Sancho and Rubio,
    J. Phys. F 15 (1985) 851): each pass folds every other lead layer into its neighbours, so
    after m passes the surface block has absorbed 2^m layers; stop when the remaining coupling
    has vanished.  Independent of the mode decomposition."""
    c = dev.contacts[k]
    adj = face_adjacency(dev, k)
    f = adj.shape[0]
    h00 = c.lead_onsite * np.eye(f) + c.lead_hopping * adj
    alpha = c.lead_hopping * np.eye(f, dtype=np.complex128)      # coupling to the next layer
    beta = alpha.copy()                                           # and back
    eps_s = h00.astype(np.complex128)
    eps = eps_s.copy()
    zi = z * np.eye(f)
    for _ in range(max_iter):
        g = np.linalg.inv(zi - eps)
        agb, bga = alpha @ g @ beta, beta @ g @ alpha
        eps_s = eps_s + agb
        eps = eps + agb + bga
        alpha = alpha @ g @ alpha
        beta = beta @ g @ beta
        if np.abs(alpha).max() + np.abs(beta).max() < tol:
            break
    else:
        raise RuntimeError("decimation did not converge")
    return (c.coupling ** 2) * np.linalg.inv(zi - eps_s)
