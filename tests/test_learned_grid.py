"""Host logic of the learned energy grid: quadrature, error estimate, proposal, features."""
import numpy as np

from paper_1702_05167_amd import learned_grid as lg


def test_trapezoid_exact_for_linear_and_error_estimate_exact_for_quadratics():
    E = np.sort(np.random.default_rng(0).uniform(-1, 2, 30))
    assert abs(lg.trapezoid(E, 3 * E - 1) - (1.5 * (E[-1] ** 2 - E[0] ** 2) - (E[-1] - E[0]))) < 1e-13
    assert np.abs(lg.interval_errors(E, 3 * E - 1)).max() < 1e-12
    # the trapezoid error of x^2 on [a, b] is (b - a)^3 / 6 for every interval
    h = np.diff(E)
    assert np.allclose(lg.interval_errors(E, E * E), h ** 3 / 6, rtol=1e-8)
    exact = (E[-1] ** 3 - E[0] ** 3) / 3
    assert abs(lg.trapezoid(E, E * E) - exact - (h ** 3 / 6).sum()) < 1e-12


def test_proposal_shape_and_ends():
    cand = np.linspace(-6, 6, 4096)
    g = np.exp(-((cand + 1) / 0.3) ** 2)
    idx = lg.proposal(cand, g, 512)
    assert idx.size == 512 and idx[0] == 0 and idx[-1] == 4095
    assert (np.diff(idx) > 0).all()
    # points crowd where the integrand curves
    inside = ((cand[idx] > -2) & (cand[idx] < 0)).sum()
    assert inside > 0.5 * 512


def test_proposal_of_flat_integrand_is_uniform():
    cand = np.linspace(0, 1, 1001)
    idx = lg.proposal(cand, np.ones(1001), 101)
    assert idx.size == 101
    assert np.abs(np.diff(idx) - 10).max() <= 1


def test_guided_grid_beats_uniform_on_a_peaked_integrand():
    # the rule itself, on a known function: same number of points, smaller trapezoid error
    cand = np.linspace(-6, 6, 4096)
    f = np.exp(-((cand - 0.5) / 0.05) ** 2) + 0.3 * np.exp(-((cand + 1.5) / 0.2) ** 2)
    exact = np.sqrt(np.pi) * (0.05 + 0.3 * 0.2)
    idx = lg.proposal(cand, f, 128)
    uni = np.arange(0, 4096, 32)
    e_g = abs(lg.trapezoid(cand[idx], f[idx]) - exact)
    e_u = abs(lg.trapezoid(cand[uni], f[uni]) - exact)
    assert e_g < e_u / 10


def test_features_and_fermi():
    X = lg.features([-6.0, 0.0, 6.0], 0.25, 32, 24)
    assert X.dtype == np.float32 and X.shape == (3, 4)
    assert np.allclose(X[:, 0], [-1, 0, 1]) and np.allclose(X[:, 1], 0.5)
    assert np.allclose(X[:, 2], 0.5) and np.allclose(X[:, 3], -0.5)
    E = np.array([-50.0, -0.1, 0.0, 0.1, 50.0])
    with np.errstate(over="ignore"):
        ref = 1.0 / (1.0 + np.exp((E - 0.05) / 0.025))
    assert np.allclose(lg.fermi(E, 0.05, 0.025), ref, rtol=1e-14, atol=1e-300)


def test_xavier_init_is_seeded_and_bounded():
    a, b = lg.xavier_init((4, 256, 256, 2), 7), lg.xavier_init((4, 256, 256, 2), 7)
    assert a.dtype == np.float32 and a.size == 67586 and np.array_equal(a, b)
    W1 = a[:1024]
    assert np.abs(W1).max() <= np.sqrt(6 / 260) and (a[1024:1280] == 0).all()
