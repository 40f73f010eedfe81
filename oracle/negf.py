"""Per-energy NEGF ingredients (oracle side; test infrastructure only).

* Lead self-energy: each contact site couples (hopping ``t_c``) to its own
  semi-infinite 1D chain (on-site ``eps0``, hopping ``t_l``).  This is the
  paper's "diagonal approximation" of the contact self-energy (operation-count
  section, SPARSE self-energy of the cuboid experiments) in closed form.
  The chain's surface Green's function g solves  t_l^2 g^2 - (z - eps0) g + 1 = 0.
  The two roots multiply to 1/t_l^2; for Im z > 0 the retarded one is the
  decaying root, |t_l g| < 1.  Sigma = t_c^2 g.
* Broadening  Gamma = i (Sigma - Sigma^dagger) = -2 Im Sigma  (diagonal Sigma).
* Lesser self-energy  Sigma^< = i (f_L Gamma_L + f_R Gamma_R)  (Eq. 2 with the
  contacts as the only source; Sigma^< is then diagonal, i.e. block diagonal
  as Algorithm 2 requires).
* Fermi function  f(E) = 1 / (1 + exp((E - mu) / kT)).
"""
from __future__ import annotations

import numpy as np


def sigma_lead(z, eps0: float, t_lead: float, t_c: float):
    """Retarded self-energy of a semi-infinite 1D chain attached by hopping t_c."""
    z = np.asarray(z, dtype=np.complex128)
    w = z - eps0
    disc = np.sqrt(w * w - 4.0 * t_lead * t_lead)
    g1 = (w + disc) / (2.0 * t_lead * t_lead)
    g2 = (w - disc) / (2.0 * t_lead * t_lead)
    g = np.where(np.abs(g1) < np.abs(g2), g1, g2)
    return (t_c * t_c) * g


def gamma_of(sig):
    """Gamma = i (Sigma - Sigma^dagger) for a diagonal Sigma."""
    return -2.0 * np.imag(sig)


def fermi(e, mu: float, kT: float):
    """Overflow-safe Fermi-Dirac occupation."""
    x = (np.asarray(e, dtype=np.float64) - mu) / kT
    out = np.empty_like(x)
    pos = x > 0
    ex = np.exp(-x[pos])
    out[pos] = ex / (1.0 + ex)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def contact_sigmas(dev, z):
    """[(sites, Sigma(z) per site)] for every contact of the device."""
    out = []
    for c in dev.contacts:
        s = complex(sigma_lead(z, c.lead_onsite, c.lead_hopping, c.coupling))
        out.append((np.asarray(c.sites, dtype=np.int64), np.full(len(c.sites), s)))
    return out


def check_symmetric(dev, tol: float = 0.0):
    """The method needs A^T = A (transposes, not adjoints, appear in Algorithm 1)."""
    h = dev.scipy_h()
    diff = abs(h - h.T).max() if h.nnz else 0.0
    if diff > tol:
        raise ValueError(f"H is not symmetric (max |H - H^T| = {diff})")
