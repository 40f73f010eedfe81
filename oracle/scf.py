"""Self-consistent NEGF-Poisson loop (oracle; test infrastructure only).

The paper names the self-consistent solution of the NEGF and Poisson equations as the setting the
method serves (abstract, Section 1) but fixes no Poisson discretisation, density formula or
mixing.  The readings used here, step by step:

* Potential energy U (one value per site) shifts the on-site entries: H -> H + diag(U).
* Electron density per site (no spin factor, hbar = 1) from the diagonal of G^< (Eq. 2):
      n_i = sum_e w_e Im G^<_ii(E_e) / (2 pi)
  with caller-supplied quadrature weights w_e over the energy grid.
* Poisson on the device grid (unit spacing, 7-point stencil), site (x, y, z) at index
  x + Nx (y + Ny z):
      sum over the three axes of (2 U_i - U_prev - U_next) = rho_i
  where a neighbour outside the device along x (the transport axis) is a lead plane, x = -1 with
  value u_left or x = Nx with value u_right (Dirichlet), and a neighbour outside along y or z is
  the site itself (zero normal derivative, Neumann).
* Source rho = c (n - n0): coupling c (e^2 / epsilon in model units), background n0.
* Linear mixing: U <- U + beta (U_new - U); residual r = max_i |U_new - U|, taken before mixing.
  Optionally Anderson mixing over the last m iterations (Anderson, J. ACM 12, 1965; the form of
  Walker and Ni, SIAM J. Numer. Anal. 49, 2011): with f_k = U_new - U_k, the differences
  dX_j = U_j+1 - U_j and dF_j = f_j+1 - f_j of the last m steps, gamma = argmin || f_k - dF gamma ||_2
  (Householder QR of dF), U_k+1 = U_k + beta f_k - (dX + beta dF) gamma; when R has a diagonal entry
  below 1e-12 of its largest the history is cleared (plain linear mixing for that step).  m = 0 is
  linear mixing.

One iteration: NEGF solve at U, density, source, Poisson solve -> U_new, residual, mix; the loop
stops after the iteration whose residual falls below tol (tol = 0: exactly `iterations` steps).
The density returned is that of the last NEGF solve (at the U before the last mixing).
"""
from __future__ import annotations

import numpy as np

from . import dense as _dense


def stencil_matrix(nx: int, ny: int, nz: int):
    """The Poisson operator as a sparse matrix (rows: sum over axes of 2 U_i minus the inside
    neighbours; an outside Neumann neighbour cancels one of the 2 U_i, an outside Dirichlet
    neighbour goes to the right-hand side)."""
    import scipy.sparse as sp
    n = nx * ny * nz
    rows, cols, vals = [], [], []
    for idx in range(n):
        x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
        diag = 0.0
        for coord, size, stride, dirichlet in ((x, nx, 1, True), (y, ny, nx, False), (z, nz, nx * ny, False)):
            for step in (-1, 1):
                c = coord + step
                if 0 <= c < size:
                    diag += 1.0
                    rows.append(idx)
                    cols.append(idx + step * stride)
                    vals.append(-1.0)
                elif dirichlet:
                    diag += 1.0
                # Neumann: the mirrored neighbour equals U_i, so the pair adds nothing
        rows.append(idx)
        cols.append(idx)
        vals.append(diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def boundary_source(nx: int, ny: int, nz: int, u_left: float, u_right: float):
    """Right-hand-side contribution of the Dirichlet lead planes."""
    b = np.zeros(nx * ny * nz)
    idx = np.arange(nx * ny * nz)
    x = idx % nx
    b[x == 0] += u_left
    b[x == nx - 1] += u_right
    return b


def poisson_solve(grid, rho, u_left: float, u_right: float):
    """U with (stencil U) = rho + lead-plane terms, by sparse direct LU."""
    import scipy.sparse.linalg as sla
    nx, ny, nz = grid
    a = stencil_matrix(nx, ny, nz).tocsc()
    return sla.spsolve(a, np.asarray(rho, dtype=np.float64) + boundary_source(nx, ny, nz, u_left, u_right))


def density(weights, gl):
    """n_i = sum_e w_e Im G^<_ii(E_e) / (2 pi)   (gl: [n_e, n] diagonals of G^<)."""
    return np.asarray(weights, dtype=np.float64) @ np.imag(np.asarray(gl)) / (2.0 * np.pi)


class Anderson:
    """Mixing of the fixed-point iteration U <- g(U): step(U, g(U)) returns the next U."""

    def __init__(self, history: int, beta: float):
        self.m, self.beta = int(history), float(beta)
        self.dX, self.dF = [], []
        self.x_prev = self.f_prev = None

    def step(self, x, gx):
        x = np.asarray(x, dtype=np.float64)
        f = np.asarray(gx, dtype=np.float64) - x
        if self.m > 0 and self.x_prev is not None:
            self.dX.append(x - self.x_prev)
            self.dF.append(f - self.f_prev)
            if len(self.dF) > self.m:
                self.dX.pop(0)
                self.dF.pop(0)
        self.x_prev, self.f_prev = x.copy(), f.copy()
        x_new = x + self.beta * f
        if self.dF:
            dF = np.stack(self.dF, axis=1)
            if dF.shape[1] > dF.shape[0]:
                # more differences than unknowns: the columns are dependent, as for a singular R
                self.dX, self.dF = [], []
                return x_new
            q, r = np.linalg.qr(dF)
            d = np.abs(np.diag(r))
            if d.min() < 1e-12 * d.max():
                self.dX, self.dF = [], []
                return x_new
            gamma = np.linalg.solve(r, q.T @ f)
            x_new = x_new - (np.stack(self.dX, axis=1) + self.beta * dF) @ gamma
        return x_new


def scf(dev, grid, energies, weights, eta, kT, mu_L, mu_R, u_left, u_right, coupling, n0=None,
        mixing=0.5, iterations=10, tol=0.0, u0=None, dense=False, history=0):
    """The loop of the module docstring on the dense oracle (dense=True: whole-face leads); returns
    u, density, residuals."""
    n = dev.n
    u = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64)
    n0 = np.zeros(n) if n0 is None else np.asarray(n0, dtype=np.float64)
    residuals = []
    dens = np.zeros(n)
    mixer = Anderson(history, mixing)
    for _ in range(iterations):
        out = _dense.solve(dev, energies, eta, kT, mu_L, mu_R, dense=dense, potential=u)
        dens = density(weights, out["gl"])
        u_new = poisson_solve(grid, coupling * (dens - n0), u_left, u_right)
        r = float(np.abs(u_new - u).max())
        residuals.append(r)
        u = mixer.step(u, u_new)
        if r < tol:
            break
    return {"u": u, "density": dens, "residuals": np.array(residuals)}
