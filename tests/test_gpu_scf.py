"""Self-consistent NEGF-Poisson loop through the C ABI: the on-site potential in the solve, the
Poisson solve, the density and the loop itself against the oracle (oracle/scf.py, oracle/dense.py).

Tolerances: Poisson and density max|x - y| <= 1e-12 max|y| (closed-form bases vs sparse LU, sums in
the same order); solves 1e-10 per energy and output vector as the other parity tests; the loop
1e-10 relative on U and the density after a fixed number of iterations (each iteration feeds the
next, so the differences of the solves carry through).
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1702_05167_amd as pkg
import paper_1702_05167_amd.hsc as H

pytestmark = pytest.mark.gpu

KW = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1)
E_MIX = np.array([-4.6, -2.1, -0.7, 0.4, 1.8, 3.3, 5.2])


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("grid", [(7, 5, 3), (1, 1, 9), (9, 1, 1), (4, 6, 1), (16, 12, 10), (32, 32, 32)])
def test_poisson_against_sparse_lu(ctx, grid):
    n = grid[0] * grid[1] * grid[2]
    rng = np.random.default_rng(n)
    rho = rng.normal(size=n)
    print(f"[poisson {grid}]", flush=True)
    u = pkg.poisson_solve(ctx, grid, torch.tensor(rho, device=ctx.torch_device), 0.35, -0.6).cpu().numpy()
    ref = oracle.scf.poisson_solve(grid, rho, 0.35, -0.6)
    assert rel(u, ref) <= 1e-12, rel(u, ref)
    # no charge: the linear lead-to-lead profile
    u0 = pkg.poisson_solve(ctx, grid, torch.zeros(n, dtype=torch.float64, device=ctx.torch_device), 0.35,
                           -0.6).cpu().numpy()
    x = np.arange(n) % grid[0]
    assert np.abs(u0 - (0.35 - 0.95 * (x + 1) / (grid[0] + 1))).max() <= 1e-13


def test_poisson_rejects_bad_grids(ctx):
    # an empty side, a non-finite lead plane, a side beyond 1024: HSC_E_ARG before any launch
    for g, ul in (((0, 2, 4), 0.0), ((2, 2, 2), float("nan")), ((2, 2, 1025), 0.0)):
        rho = torch.zeros(g[0] * g[1] * g[2], dtype=torch.float64, device=ctx.torch_device)
        with pytest.raises(H.HscError) as e:
            pkg.poisson_solve(ctx, g, rho, ul, 0.0)
        assert e.value.code == -1


def test_density_against_oracle(ctx):
    rng = np.random.default_rng(3)
    ne, n = 17, 1000
    gl = rng.normal(size=(ne, n)) + 1j * rng.normal(size=(ne, n))
    w = rng.uniform(0.1, 1.0, ne)
    d = pkg.density(ctx, torch.tensor(w, device=ctx.torch_device), torch.tensor(gl, device=ctx.torch_device))
    ref = oracle.scf.density(w, gl)
    assert rel(d.cpu().numpy(), ref) <= 1e-13


def _solve(ctx, dev, E, precision, potential, leaf=2, dense=False, **kw):
    tree = pkg.Tree.from_device(dev, leaf_side=leaf, dense=dense)
    pot = torch.tensor(potential, device=ctx.torch_device) if potential is not None else None
    out = pkg.solve(ctx, tree, torch.tensor(E, device=ctx.torch_device),
                    want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS, precision=precision, potential=pot,
                    **{**KW, **kw})
    return tree, {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("precision,eta", [(0, 0.05), (1, 0.05), (2, 1e-8), (3, 1e-8)])
def test_solve_with_potential_against_oracle(ctx, precision, eta):
    dev = synth.cuboid(6, 5, 4, onsite=np.random.default_rng(8).normal(0, 0.3, 120))
    U = np.random.default_rng(9).uniform(-0.6, 0.6, 120)
    print(f"[potential precision {precision}]", flush=True)
    _, g = _solve(ctx, dev, E_MIX, precision, U, eta=eta)
    ref = oracle.dense.solve(dev, E_MIX, potential=U, **{**KW, "eta": eta})
    for e in range(len(E_MIX)):
        for k in ("gr", "gl"):
            assert rel(g[k][e], ref[k][e]) <= 1e-10, (k, E_MIX[e])
        assert abs(g["trans"][e] - ref["trans"][e]) <= 1e-10 * max(ref["trans"][e], 1e-12)
    assert (g["status"] == 0).all()


def test_potential_is_cleared_and_graph_replays_it(ctx):
    # a later call without U solves H itself again (the plan's potential is zeroed), and graph
    # replay reads the potential of each call
    dev = synth.cuboid(7, 4, 4, onsite=np.random.default_rng(1).normal(0, 0.3, 112))
    U = np.linspace(0.4, -0.4, 112)
    tree = pkg.Tree.from_device(dev, leaf_side=2)
    E = torch.tensor(E_MIX, device=ctx.torch_device)
    want = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL
    plain = pkg.solve(ctx, tree, E, want=want, **KW)["gr"].cpu().numpy()
    pot = torch.tensor(U, device=ctx.torch_device)
    with_u = pkg.solve(ctx, tree, E, want=want, potential=pot, **KW)["gr"].cpu().numpy()
    again = pkg.solve(ctx, tree, E, want=want, **KW)["gr"].cpu().numpy()
    assert np.array_equal(plain, again)
    assert rel(with_u, oracle.dense.solve(dev, E_MIX, potential=U, **KW)["gr"]) <= 1e-10
    g1 = pkg.solve(ctx, tree, E, want=want, potential=pot, graph=1, batch=4, **KW)["gr"].cpu().numpy()
    g2 = pkg.solve(ctx, tree, E, want=want, potential=-pot, graph=1, batch=4, **KW)["gr"].cpu().numpy()
    assert rel(g1, with_u) <= 1e-13
    assert rel(g2, oracle.dense.solve(dev, E_MIX, potential=-U, **KW)["gr"]) <= 1e-10


def test_whole_face_contacts_with_potential(ctx):
    dev = synth.cuboid(6, 4, 4, onsite=np.random.default_rng(6).normal(0, 0.3, 96))
    U = np.random.default_rng(7).uniform(-0.3, 0.5, 96)
    _, g = _solve(ctx, dev, E_MIX, 3, U, dense=True)
    ref = oracle.dense.solve(dev, E_MIX, dense=True, potential=U, **KW)
    for e in range(len(E_MIX)):
        assert rel(g["gr"][e], ref["gr"][e]) <= 1e-10 and rel(g["gl"][e], ref["gl"][e]) <= 1e-10


def test_batch_rejects_a_potential(ctx):
    dev = synth.cuboid(4, 3, 3)
    trees = [pkg.Tree.from_device(dev, leaf_side=2), pkg.Tree.from_device(dev, leaf_side=2)]
    E = torch.tensor(E_MIX[:2], device=ctx.torch_device)
    pot = torch.zeros(36, dtype=torch.float64, device=ctx.torch_device)
    opts = H.SolveOpts(1e-8, 0.025, 0.1, -0.1, pkg.HSC_DIAG_GR, 0, 0.0, 0, 3, 0, 0, 0, 0, C.c_void_p(pot.data_ptr()))
    out = [torch.empty((2, 36), dtype=torch.complex128, device=ctx.torch_device) for _ in trees]
    th = (C.c_void_p * 2)(*[t.h.value for t in trees])
    ne = np.array([2, 2], np.int32)
    ea = (C.c_void_p * 2)(E.data_ptr(), E.data_ptr())
    gr = (C.c_void_p * 2)(*[o.data_ptr() for o in out])
    rc = H.lib().hsc_solve_batch(ctx.h, 2, th, H._ptr(ne), ea, C.byref(opts), gr, None, None, None, None, None)
    assert rc == -1


SCF_DEV = dict(shape=(5, 4, 3), seed=12)


def _scf_case():
    nx, ny, nz = SCF_DEV["shape"]
    n = nx * ny * nz
    dev = synth.cuboid(nx, ny, nz, onsite=np.random.default_rng(SCF_DEV["seed"]).normal(0, 0.2, n))
    E = np.linspace(-6.0, 2.0, 25)
    w = np.full(25, E[1] - E[0])
    w[0] = w[-1] = 0.5 * w[0]
    return dev, (nx, ny, nz), E, w


@pytest.mark.parametrize("precision,coupling,mixing", [(2, 0.2, 0.4), (3, 0.2, 0.4), (3, 0.3, 0.7)])
def test_scf_iterations_against_oracle(ctx, precision, coupling, mixing):
    # four iterations of the loop with a bias between the lead planes and a background charge; with
    # coupling 0.3 and mixing 0.7 the third iteration overshoots by several units of energy (the
    # loop recovers later), which takes the solves far from the starting potential
    dev, grid, E, w = _scf_case()
    n = dev.n
    n0 = np.full(n, 0.02)
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.1, mu_R=-0.1)
    tree = pkg.Tree.from_device(dev, leaf_side=2)
    print(f"[scf precision {precision}]", flush=True)
    u, dens, res = pkg.scf(ctx, tree, grid, E, w, u_left=0.1, u_right=-0.1, coupling=coupling, n0=n0,
                           mixing=mixing, max_iter=4, precision=precision, **kw)
    ref = oracle.scf.scf(dev, grid, E, w, u_left=0.1, u_right=-0.1, coupling=coupling, n0=n0, mixing=mixing,
                         iterations=4, **kw)
    print("scf residuals", res, ref["residuals"])
    assert len(res) == 4
    assert rel(u.cpu().numpy(), ref["u"]) <= 1e-10
    assert rel(dens.cpu().numpy(), ref["density"]) <= 1e-10
    assert np.abs(res - ref["residuals"]).max() <= 1e-10 * ref["residuals"].max()


def test_scf_with_whole_face_leads_against_oracle(ctx):
    # three iterations on a 5 x 4 x 3 device whose contacts are whole faces (dense self-energies)
    dev, grid, E, w = _scf_case()
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.1, mu_R=-0.1)
    tree = pkg.Tree.from_device(dev, leaf_side=2, dense=True)
    u, dens, res = pkg.scf(ctx, tree, grid, E, w, u_left=0.1, u_right=-0.1, coupling=0.2, mixing=0.4, max_iter=3,
                           **kw)
    ref = oracle.scf.scf(dev, grid, E, w, u_left=0.1, u_right=-0.1, coupling=0.2, mixing=0.4, iterations=3,
                         dense=True, **kw)
    print("scf whole-face residuals", res, ref["residuals"])
    assert rel(u.cpu().numpy(), ref["u"]) <= 1e-10
    assert rel(dens.cpu().numpy(), ref["density"]) <= 1e-10


def test_scf_converges_to_a_fixed_point(ctx):
    # run to a tolerance on a 6 x 5 x 4 device; the converged U solves Poisson with the density it
    # produces, checked with the oracle's sparse Poisson solve on the GPU density
    nx, ny, nz = 6, 5, 4
    n = nx * ny * nz
    dev = synth.cuboid(nx, ny, nz, onsite=np.random.default_rng(4).normal(0, 0.2, n))
    E = np.linspace(-6.0, 2.0, 33)
    w = np.full(33, E[1] - E[0])
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.05, mu_R=-0.05)
    tree = pkg.Tree.from_device(dev, leaf_side=3)
    u, dens, res = pkg.scf(ctx, tree, (nx, ny, nz), E, w, coupling=0.2, mixing=0.6, max_iter=60, tol=1e-11, **kw)
    print("scf residuals", res)
    assert res[-1] < 1e-11 and len(res) < 60 and res[-1] < 1e-6 * res[0]
    u = u.cpu().numpy()
    g = pkg.solve(ctx, tree, torch.tensor(E, device=ctx.torch_device), want=pkg.HSC_DIAG_GL,
                  potential=torch.tensor(u, device=ctx.torch_device), **kw)["gl"].cpu().numpy()
    d = oracle.scf.density(w, g)
    assert np.abs(oracle.scf.poisson_solve((nx, ny, nz), 0.2 * d, 0.0, 0.0) - u).max() < 1e-10


@pytest.mark.parametrize("history", [1, 4])
def test_scf_anderson_iterations_against_oracle(ctx, history):
    # six iterations with Anderson mixing over the last `history` steps: the device keeps the
    # differences, the host solves the small least-squares problem, and the update runs on the device
    dev, grid, E, w = _scf_case()
    n0 = np.full(dev.n, 0.02)
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.1, mu_R=-0.1)
    tree = pkg.Tree.from_device(dev, leaf_side=2)
    print(f"[scf anderson history {history}]", flush=True)
    u, dens, res = pkg.scf(ctx, tree, grid, E, w, u_left=0.1, u_right=-0.1, coupling=0.2, n0=n0, mixing=0.4,
                           max_iter=6, history=history, **kw)
    ref = oracle.scf.scf(dev, grid, E, w, u_left=0.1, u_right=-0.1, coupling=0.2, n0=n0, mixing=0.4,
                         iterations=6, history=history, **kw)
    print("scf anderson residuals", res, ref["residuals"])
    assert len(res) == 6
    assert rel(u.cpu().numpy(), ref["u"]) <= 1e-10
    assert rel(dens.cpu().numpy(), ref["density"]) <= 1e-10
    assert np.abs(res - ref["residuals"]).max() <= 1e-10 * ref["residuals"].max()


def test_scf_anderson_with_more_history_than_sites(ctx):
    # a three-site chain with a history of five: the fifth iteration holds four differences of three
    # unknowns, which both sides treat as dependent (a linear step, history restarted)
    dev = synth.cuboid(3, 1, 1, onsite=np.array([0.1, -0.2, 0.05]))
    E = np.linspace(-3.0, 1.0, 17)
    w = np.full(17, E[1] - E[0])
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.1, mu_R=-0.1)
    tree = pkg.Tree.from_device(dev, leaf_side=2)
    u, dens, res = pkg.scf(ctx, tree, (3, 1, 1), E, w, u_left=0.1, u_right=-0.1, coupling=0.3, mixing=0.5,
                           max_iter=8, history=5, **kw)
    ref = oracle.scf.scf(dev, (3, 1, 1), E, w, u_left=0.1, u_right=-0.1, coupling=0.3, mixing=0.5, iterations=8,
                         history=5, **kw)
    print("tiny anderson residuals", res, ref["residuals"])
    assert len(res) == 8
    assert rel(u.cpu().numpy(), ref["u"]) <= 1e-10
    assert np.abs(res - ref["residuals"]).max() <= 1e-10 * ref["residuals"].max()


def test_scf_anderson_reaches_the_linear_fixed_point_sooner(ctx):
    # on a 4 x 3 x 3 device, linear mixing needs about three times the iterations of Anderson mixing
    # over four steps to reach a residual of 1e-12; both stop at the same potential
    nx, ny, nz = 4, 3, 3
    n = nx * ny * nz
    dev = synth.cuboid(nx, ny, nz, onsite=np.random.default_rng(5).normal(0, 0.2, n))
    E = np.linspace(-6.0, 2.0, 33)
    w = np.full(33, E[1] - E[0])
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.05, mu_R=-0.05, coupling=0.2, mixing=0.6, max_iter=60, tol=1e-12)
    tree = pkg.Tree.from_device(dev, leaf_side=2)
    u_lin, _, r_lin = pkg.scf(ctx, tree, (nx, ny, nz), E, w, **kw)
    u_acc, _, r_acc = pkg.scf(ctx, tree, (nx, ny, nz), E, w, history=4, **kw)
    print("linear", len(r_lin), r_lin[-1], "anderson", len(r_acc), r_acc[-1])
    assert r_lin[-1] < 1e-12 and r_acc[-1] < 1e-12 and len(r_lin) < 60
    assert 2 * len(r_acc) <= len(r_lin)
    assert np.abs(u_lin.cpu().numpy() - u_acc.cpu().numpy()).max() < 1e-11
    assert u_lin.shape == (n,)


def test_scf_rejects_a_grid_that_is_not_the_tree(ctx):
    dev, grid, E, w = _scf_case()
    tree = pkg.Tree.from_device(dev, leaf_side=2)
    with pytest.raises(H.HscError) as e:
        pkg.scf(ctx, tree, (grid[0], grid[1], grid[2] + 1), E, w, coupling=0.1, max_iter=1)
    assert e.value.code == -1
    with pytest.raises(H.HscError):
        pkg.scf(ctx, tree, grid, E, w, coupling=0.1, mixing=1.5, max_iter=1)
    for history in (-1, 17):
        with pytest.raises(H.HscError):
            pkg.scf(ctx, tree, grid, E, w, coupling=0.1, max_iter=1, history=history)
    # the binding checks lengths before any call: weights per energy, a start potential per site
    with pytest.raises(ValueError):
        pkg.scf(ctx, tree, grid, E, w[:-1], coupling=0.1, max_iter=1)
    with pytest.raises(ValueError):
        pkg.scf(ctx, tree, grid, E, w, coupling=0.1, max_iter=1, u0=np.zeros(dev.n + 1))
    with pytest.raises(ValueError):
        pkg.density(ctx, torch.ones(2, dtype=torch.float64, device=ctx.torch_device),
                    torch.zeros((2, dev.n), dtype=torch.complex64, device=ctx.torch_device))
