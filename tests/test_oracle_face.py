"""Pins of the oracle's DENSE contact self-energy (whole-face leads, Section 3.1.2's DENSE case)
against facts that do not come from the oracle's own formula."""
import numpy as np
import pytest

import synth
import oracle
from oracle.face import face_sigma, decimation, face_adjacency, normal_axis
from oracle.negf import sigma_lead


def _lead_h00(dev, k):
    c = dev.contacts[k]
    adj = face_adjacency(dev, k)
    return c.lead_onsite * np.eye(len(adj)) + c.lead_hopping * adj


@pytest.mark.parametrize("shape", [(4, 5, 3), (3, 1, 6), (6, 7, 7)])
@pytest.mark.parametrize("energy", [-5.1, -2.3, -0.4, 0.9, 3.7, 6.8])
def test_surface_dyson_equation(shape, energy):
    # g_s = Sigma / t_c^2 solves g = (z - H00 - H01 g H01^T)^-1 with H01 = t_l I, and is the
    # retarded solution: Gamma = i (Sigma - Sigma^dagger) is positive semidefinite
    dev = synth.cuboid(*shape)
    z = energy + 1e-8j
    for k in (0, 1):
        c = dev.contacts[k]
        sig, _ = face_sigma(dev, k, z)
        g = sig / c.coupling ** 2
        h00 = _lead_h00(dev, k)
        lhs = g @ (z * np.eye(len(g)) - h00 - c.lead_hopping ** 2 * g)
        assert np.abs(lhs - np.eye(len(g))).max() < 1e-11
        gam = 1j * (sig - sig.conj().T)
        assert np.abs(gam.imag).max() < 1e-14
        assert np.linalg.eigvalsh(gam.real).min() > -1e-12
        assert np.abs(sig - sig.T).max() < 1e-14


@pytest.mark.parametrize("energy", [-4.4, -1.7, 0.35, 2.9])
def test_decimation_agrees(energy):
    # Sancho-Rubio decimation (an iteration over lead layers, no mode decomposition)
    dev = synth.cuboid(3, 5, 4)
    dev.contacts[1].lead_onsite = 0.3
    dev.contacts[1].coupling = -0.7
    for k in (0, 1):
        z = energy + 1e-6j
        sig, _ = face_sigma(dev, k, z)
        sd = decimation(dev, k, z)
        assert np.abs(sig - sd).max() < 1e-9 * np.abs(sig).max()


def test_one_site_face_is_the_chain():
    dev = synth.chain(5)
    for energy in (-2.5, -0.3, 1.1, 3.0):
        z = energy + 1e-8j
        sig, v = face_sigma(dev, 0, z)
        assert sig.shape == (1, 1)
        assert abs(sig[0, 0] - complex(sigma_lead(z, 0.0, -1.0, -1.0))) < 1e-15
    # so on a chain the dense and the per-site (diagonal) self-energies solve the same problem
    e = [-1.5, 0.2, 1.9, 2.4]
    a = oracle.dense.solve(dev, e, 1e-8, 0.025, 0.1, -0.1)
    b = oracle.dense.solve(dev, e, 1e-8, 0.025, 0.1, -0.1, dense=True)
    for key in ("gr", "gl", "a_l", "a_r", "trans"):
        assert np.allclose(a[key], b[key], rtol=1e-13, atol=1e-15), key


@pytest.mark.parametrize("shape", [(5, 4, 3), (2, 6, 5), (7, 3, 1)])
def test_clean_wire_counts_open_modes(shape):
    # a clean device with the lead's own parameters is a piece of an infinite perfect wire: each
    # transverse mode with |E - eps - t_l mu_m| < 2 |t_l| carries exactly one unit of transmission
    dev = synth.cuboid(*shape)
    mu = np.linalg.eigvalsh(face_adjacency(dev, 0))
    lam = -1.0 * mu
    energies = []
    for energy in np.linspace(-6.5, 6.5, 53):
        edges = np.concatenate([lam - 2.0, lam + 2.0])
        if np.abs(edges - energy).min() > 0.05:
            energies.append(energy)
    out = oracle.dense.solve(dev, energies, 1e-12, 0.025, 0.1, -0.1, dense=True)
    for energy, t in zip(energies, out["trans"]):
        count = int(np.sum(np.abs(energy - lam) < 2.0))
        assert abs(t - count) < 1e-6, (energy, t, count)


@pytest.mark.parametrize("energy", [-3.2, -0.8, 0.45, 2.6])
def test_dense_sum_rule_and_left_face_trace(energy):
    # i (G - G^dagger) = G (Gamma_L + Gamma_R + 2 eta) G^dagger, diagonal part; and the
    # transmission equals the left-face trace Tr(Gamma_L A_R) taken over the face block
    dev = synth.cuboid(5, 4, 4, onsite=np.random.default_rng(3).normal(0, 0.3, 80))
    eta = 1e-3
    out = oracle.dense.solve(dev, [energy], eta, 0.025, 0.1, -0.1, dense=True)
    lhs = -2.0 * out["gr"][0].imag
    rhs = out["a_l"][0] + out["a_r"][0] + out["a_eta"][0]
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-14)
    z = energy + 1j * eta
    g = oracle.dense.green(dev, energy, eta, dense=True)
    ls = np.asarray(dev.contacts[0].sites)
    rs = np.asarray(dev.contacts[1].sites)
    s_l, _ = face_sigma(dev, 0, z)
    s_r, _ = face_sigma(dev, 1, z)
    gam_l = (1j * (s_l - s_l.conj().T)).real
    gam_r = (1j * (s_r - s_r.conj().T)).real
    a_r_full = g[:, rs] @ gam_r @ g[:, rs].conj().T
    t_face = np.sum(gam_l * a_r_full[np.ix_(ls, ls)].real)
    assert abs(t_face - out["trans"][0]) < 1e-11 * max(1.0, out["trans"][0])
    # reciprocity
    a_l_full = g[:, ls] @ gam_l @ g[:, ls].conj().T
    t_rl = np.sum(gam_r * a_l_full[np.ix_(rs, rs)].real)
    assert abs(t_rl - out["trans"][0]) < 1e-11 * max(1.0, out["trans"][0])


@pytest.mark.parametrize("energy", [-2.9, -0.6, 1.3])
def test_dense_rgf_matches_definition(energy):
    # slab recursion (Section 2.1) with the dense face blocks against the dense inverse
    dev = synth.cuboid(6, 4, 3, onsite=np.random.default_rng(9).normal(0, 0.3, 72))
    a = oracle.dense.solve(dev, [energy], 1e-8, 0.025, 0.1, -0.1, dense=True)
    b = oracle.rgf.solve(dev, [energy], 1e-8, 0.025, 0.1, -0.1, dense=True)
    for key in ("gr", "gl", "a_l", "a_r", "trans"):
        scale = np.abs(a[key]).max()
        assert np.abs(a[key] - b[key]).max() < 1e-10 * scale, key


def test_normal_axis_and_rejection():
    dev = synth.cuboid(4, 3, 2)
    assert normal_axis(dev) == 0
    bad = synth.cuboid(4, 3, 2)
    bad.contacts[1].sites = np.array([1, 2])       # not a flat face parallel to the left one
    bad.contacts[0].sites = np.array([0, 4])
    with pytest.raises(ValueError):
        normal_axis(bad)
