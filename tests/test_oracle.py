"""Pins of the CPU oracle against closed forms, invariants and independent routes.

Nothing here compares the oracle with itself: every expected value comes from
a formula derived independently of the oracle's code path (a 1D chain solved
in closed form, a transverse-mode decomposition, textbook lead self-energy),
or from a mathematical identity the exact answer must satisfy.
"""
import numpy as np
import pytest

import synth
import oracle
from oracle.negf import sigma_lead, gamma_of, fermi

ETA = 1e-8
KT, MUL, MUR = 0.025, 0.1, -0.1


# ---- lead self-energy ---------------------------------------------------------------------

@pytest.mark.parametrize("t", [-1.0, -2.7, 0.8])
def test_sigma_quadratic_and_retarded_branch(t):
    E = np.linspace(-3 * abs(t), 3 * abs(t), 121)
    z = E + 1j * ETA
    s = sigma_lead(z, 0.0, t, t)
    # S solves S^2 - z S + t^2 = 0 (surface Green's function of the chain times t^2)
    assert np.abs(s * s - z * s + t * t).max() <= 1e-13 * t * t
    assert (s.imag <= 0).all()                        # retarded: Gamma >= 0
    assert (np.abs(s) < abs(t) + 1e-12).all()         # decaying root


def test_sigma_textbook_in_band_and_out_of_band():
    t = -1.0
    E = np.linspace(-1.99, 1.99, 41)
    s = sigma_lead(E + 1j * 1e-14, 0.0, t, t)
    # in band: Sigma = E/2 - i sqrt(4 t^2 - E^2)/2
    ref = E / 2 - 0.5j * np.sqrt(4 * t * t - E * E)
    assert np.abs(s - ref).max() < 1e-9
    Eo = np.array([-5.0, -2.5, 2.5, 5.0])
    so = sigma_lead(Eo + 1j * 1e-14, 0.0, t, t)
    # out of band: real, Sigma = (E - sign(E) sqrt(E^2 - 4t^2))/2
    refo = (Eo - np.sign(Eo) * np.sqrt(Eo * Eo - 4 * t * t)) / 2
    assert np.abs(so - refo).max() < 1e-9


def test_sigma_coupling_and_onsite_scaling():
    z = 0.37 + 1e-8j
    base = sigma_lead(z - 0.2, 0.0, -1.3, -1.3)
    shifted = sigma_lead(z, 0.2, -1.3, -1.3)
    assert abs(base - shifted) < 1e-14
    assert abs(sigma_lead(z - 0.2, 0.0, -1.3, -0.5) - base * (0.5 / 1.3) ** 2) < 1e-14


def test_fermi():
    assert fermi(np.array([0.3]), 0.3, 0.025)[0] == 0.5
    x = np.linspace(-2, 2, 41)
    assert np.abs(fermi(0.1 + x, 0.1, 0.025) + fermi(0.1 - x, 0.1, 0.025) - 1).max() < 1e-15
    big = fermi(np.array([-1e4, 1e4]), 0.0, 0.025)
    assert big[0] == 1.0 and big[1] == 0.0
    y = np.linspace(-0.2, 0.2, 9)
    assert np.abs(fermi(y, 0.0, 0.025) - 1 / (1 + np.exp(y / 0.025))).max() < 1e-15


# ---- 1D chain in closed form ----------------------------------------------------------------

def chain_closed_form(m, E, eta=ETA, t=-1.0):
    """Device = M sites of an infinite chain: G_ij = g lam^|i-j|, g = 1/(z - 2 Sigma), lam = Sigma/t."""
    z = E + 1j * eta
    s = sigma_lead(z, 0.0, t, t)
    g = 1.0 / (z - 2 * s)
    lam = s / t
    gam = gamma_of(s)
    i = np.arange(m)
    G = g * lam ** np.abs(i[:, None] - i[None, :])
    return G, gam


@pytest.mark.parametrize("E", [-1.7, -0.4, 0.0, 0.9, 1.5, -2.6, 3.1])
def test_chain_against_closed_form(E):
    m = 23
    dev = synth.chain(m)
    G, gam = chain_closed_form(m, E)
    a_l = gam * np.abs(G[:, 0]) ** 2
    a_r = gam * np.abs(G[:, m - 1]) ** 2
    T = gam * gam * np.abs(G[0, m - 1]) ** 2
    gl = 1j * (fermi(np.array([E]), MUL, KT)[0] * a_l + fermi(np.array([E]), MUR, KT)[0] * a_r)
    for mod in (oracle.dense, oracle.rgf):
        out = mod.solve(dev, [E], ETA, KT, MUL, MUR)
        assert np.abs(out["gr"][0] - np.diag(G)).max() <= 1e-12 * np.abs(G).max()
        assert np.abs(out["a_l"][0] - a_l).max() <= 1e-12 * max(a_l.max(), 1e-300)
        assert np.abs(out["a_r"][0] - a_r).max() <= 1e-12 * max(a_r.max(), 1e-300)
        assert abs(out["trans"][0] - T) <= 1e-12 * max(T, 1e-300) + 1e-300
        assert np.abs(out["gl"][0] - gl).max() <= 1e-12 * max(np.abs(gl).max(), 1e-300)
    sm = oracle.sampled.solve_sites(dev, [E], ETA, KT, MUL, MUR, np.arange(m), want_trans=True)
    assert np.abs(sm["gr"][0] - np.diag(G)).max() <= 1e-12 * np.abs(G).max()
    assert abs(sm["trans"][0] - T) <= 1e-12 * max(T, 1e-300) + 1e-300


def test_chain_unit_in_band_transmission():
    # in the lead band a clean chain transmits one channel: T = 1 - O(M eta / v)
    m = 40
    dev = synth.chain(m)
    E = np.linspace(-1.8, 1.8, 13)
    out = oracle.dense.solve(dev, E, ETA, KT, MUL, MUR)
    assert np.abs(out["trans"] - 1).max() < 1e-5
    out = oracle.dense.solve(dev, E, 1e-13, KT, MUL, MUR)
    assert np.abs(out["trans"] - 1).max() < 1e-10


# ---- clean cuboid: transverse-mode decomposition --------------------------------------------

def cuboid_modes(nx, ny, nz, E, eta=ETA, t=-1.0):
    """Hard-wall sine modes across (y, z); each mode is an independent 1D problem along x."""
    z = E + 1j * eta
    s = sigma_lead(z, 0.0, t, t)
    gam = gamma_of(s)
    py = np.arange(1, ny + 1)
    pz = np.arange(1, nz + 1)
    phy = np.sqrt(2.0 / (ny + 1)) * np.sin(np.pi * np.outer(np.arange(ny) + 1, py) / (ny + 1))   # [y, my]
    phz = np.sqrt(2.0 / (nz + 1)) * np.sin(np.pi * np.outer(np.arange(nz) + 1, pz) / (nz + 1))
    ey = 2 * t * np.cos(np.pi * py / (ny + 1))
    ez = 2 * t * np.cos(np.pi * pz / (nz + 1))
    n = nx * ny * nz
    gr = np.zeros(n, complex)
    a_l = np.zeros(n)
    a_r = np.zeros(n)
    T = 0.0
    hx = np.diag(np.full(nx - 1, t), 1) + np.diag(np.full(nx - 1, t), -1)
    idx = np.arange(n)
    xs, ys, zs = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    for my in range(ny):
        for mz in range(nz):
            a = (z - ey[my] - ez[mz]) * np.eye(nx) - hx
            a[0, 0] -= s
            a[nx - 1, nx - 1] -= s
            gx = np.linalg.inv(a)
            w = (phy[ys, my] * phz[zs, mz]) ** 2
            gr += gx[xs, xs] * w
            a_l += gam * np.abs(gx[xs, 0]) ** 2 * w
            a_r += gam * np.abs(gx[xs, nx - 1]) ** 2 * w
            T += gam * gam * abs(gx[0, nx - 1]) ** 2
    return gr, a_l, a_r, T


@pytest.mark.parametrize("E", [-4.1, -1.2, 0.3, 2.2])
def test_clean_cuboid_against_modes(E):
    nx, ny, nz = 7, 5, 4
    dev = synth.cuboid(nx, ny, nz)
    gr, a_l, a_r, T = cuboid_modes(nx, ny, nz, E)
    for mod in (oracle.dense, oracle.rgf):
        out = mod.solve(dev, [E], ETA, KT, MUL, MUR)
        assert np.abs(out["gr"][0] - gr).max() <= 1e-11 * np.abs(gr).max()
        assert np.abs(out["a_l"][0] - a_l).max() <= 1e-11 * max(a_l.max(), 1e-300)
        assert np.abs(out["a_r"][0] - a_r).max() <= 1e-11 * max(a_r.max(), 1e-300)
        assert abs(out["trans"][0] - T) <= 1e-11 * max(T, 1e-12)


# ---- invariants on a disordered device -------------------------------------------------------

@pytest.fixture(scope="module")
def disordered():
    rng = np.random.default_rng(5)
    dev = synth.cuboid(6, 5, 4, onsite=rng.uniform(-0.5, 0.5, 120))
    return dev


@pytest.mark.parametrize("E", [-4.6, -1.9, -0.2, 0.8, 2.7])
def test_invariants(disordered, E):
    dev = disordered
    G = oracle.dense.green(dev, E, ETA)
    out = oracle.dense.solve(dev, [E], ETA, KT, MUL, MUR)
    scale = np.abs(G).max()
    assert np.abs(G - G.T).max() <= 1e-12 * scale                        # A^T = A  ->  G^T = G
    assert (out["gr"][0].imag <= 1e-12 * scale).all()                    # retarded: Im G_ii <= 0
    # i (G - G^dag) = G (Gamma_L + Gamma_R + 2 eta) G^dag, diagonal
    lhs = -2 * out["gr"][0].imag
    rhs = out["a_l"][0] + out["a_r"][0] + out["a_eta"][0]
    assert np.abs(lhs - rhs).max() <= 1e-12 * max(lhs.max(), 1e-300)
    # reciprocity Tr Gamma_L A_R = Tr Gamma_R A_L
    z = E + 1j * ETA
    (ls, sl), (rs, sr) = oracle.negf.contact_sigmas(dev, z)
    t_lr = gamma_of(sl) @ out["a_r"][0][ls]
    t_rl = gamma_of(sr) @ out["a_l"][0][rs]
    assert abs(t_lr - t_rl) <= 1e-12 * max(t_lr, 1e-300) + 1e-300
    assert abs(out["trans"][0] - t_lr) <= 1e-12 * max(t_lr, 1e-300) + 1e-300
    # lesser function: anti-Hermitian diagonal, -i G^< >= 0, bounded transmission
    gl = out["gl"][0]
    assert np.abs(gl.real).max() <= 1e-12 * max(np.abs(gl).max(), 1e-300)
    assert (gl.imag >= -1e-12 * max(np.abs(gl).max(), 1e-300)).all()
    assert -1e-12 <= out["trans"][0] <= min(len(ls), len(rs)) + 1e-9


@pytest.mark.parametrize("E", [-5.3, -2.2, -0.6, 1.1, 3.4])
def test_rgf_and_sampled_match_dense(disordered, E):
    dev = disordered
    a = oracle.dense.solve(dev, [E], ETA, KT, MUL, MUR)
    b = oracle.rgf.solve(dev, [E], ETA, KT, MUL, MUR)
    sites = np.array([0, 7, 33, 64, 119])
    c = oracle.sampled.solve_sites(dev, [E], ETA, KT, MUL, MUR, sites, want_trans=True)
    for k in ("gr", "gl", "a_l", "a_r"):
        sc = np.abs(a[k][0]).max()
        assert np.abs(a[k][0] - b[k][0]).max() <= 1e-11 * sc
        assert np.abs(a[k][0][sites] - c[k][0]).max() <= 1e-11 * sc
    assert abs(a["trans"][0] - b["trans"][0]) <= 1e-11 * max(a["trans"][0], 1e-12)
    assert abs(a["trans"][0] - c["trans"][0]) <= 1e-11 * max(a["trans"][0], 1e-12)


def test_trilayer_rgf_matches_dense():
    dev = synth.trilayer(8, 7)
    E = [-2.1, 0.35, 2.6]
    a = oracle.dense.solve(dev, E, ETA, KT, MUL, MUR)
    b = oracle.rgf.solve(dev, E, ETA, KT, MUL, MUR)
    for k in ("gr", "gl", "a_l", "a_r"):
        sc = np.abs(a[k]).max()
        assert np.abs(a[k] - b[k]).max() <= 1e-11 * sc
    assert np.abs(a["trans"] - b["trans"]).max() <= 1e-11 * max(a["trans"].max(), 1e-12)


def test_hamiltonian_builders_are_symmetric():
    for dev in (synth.config0_device(), synth.trilayer(9, 6), synth.cuboid(3, 4, 5)):
        oracle.negf.check_symmetric(dev)
        h = dev.scipy_h()
        assert (abs(h - h.conj().T)).max() == 0          # real symmetric (Hermitian too)


def _bond_pairs(dev):
    h = dev.scipy_h().tocoo()
    m = h.row < h.col
    return np.unique(np.stack([h.row[m], h.col[m]], 1), axis=0)


@pytest.mark.parametrize("dense", [False, True])
def test_bond_lesser_continuity(dense):
    # steady state: at a site with no lead, sum_j (H_ij G^<_ji - G^<_ij H_ji) = 2 i eta G^<_ii
    # (the eta broadening is the only sink) -- an identity of the Dyson equation, independent of
    # how G^< is formed
    rng = np.random.default_rng(5)
    dev = synth.cuboid(5, 4, 3, onsite=rng.normal(0, 0.3, 60))
    eta = 1e-3
    pairs = _bond_pairs(dev)
    E = [-1.3, 0.4, 2.2]
    b = oracle.dense.bonds(dev, E, eta, 0.025, 0.3, -0.2, pairs, dense=dense)
    d = oracle.dense.solve(dev, E, eta, 0.025, 0.3, -0.2, dense=dense)
    h = dev.dense_h()
    contact = set(np.concatenate([c.sites for c in dev.contacts]).tolist())
    for e in range(len(E)):
        gl = np.zeros((dev.n, dev.n), np.complex128)
        gl[pairs[:, 0], pairs[:, 1]] = b["gl"][e]
        gl[pairs[:, 1], pairs[:, 0]] = -np.conj(b["gl"][e])           # anti-Hermitian
        gl[np.arange(dev.n), np.arange(dev.n)] = d["gl"][e]
        lhs = np.diag(h @ gl - gl @ h)
        for s in range(dev.n):
            if s in contact:
                continue
            assert abs(lhs[s] - 2j * eta * gl[s, s]) < 1e-12 * np.abs(gl).max(), (s, lhs[s])


def test_bond_lesser_equilibrium():
    # equal occupations: G^< = f (G^a - G^r) - 2 eta f G G^dagger; with eta -> 0 the bond entries
    # of G^< follow from those of G^r alone (G symmetric): G^<_ij = -2 i f Im G^r_ij
    rng = np.random.default_rng(6)
    dev = synth.cuboid(6, 3, 3, onsite=rng.normal(0, 0.3, 54))
    pairs = _bond_pairs(dev)
    E = [-1.7, -0.2, 1.1]
    b = oracle.dense.bonds(dev, E, 1e-12, 0.025, 0.05, 0.05, pairs)
    f = oracle.negf.fermi(np.array(E), 0.05, 0.025)
    for e in range(len(E)):
        ref = -2j * f[e] * b["gr"][e].imag
        assert np.abs(b["gl"][e] - ref).max() < 1e-9 * max(np.abs(ref).max(), 1e-300)
