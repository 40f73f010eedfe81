"""Learned energy grid: a surrogate network chooses the energies of the charge integral.

The electron count of a device is Q = integral dE n(E), n(E) = (1/2pi) sum_i -i G^<_ii(E)
(hbar = 1, no spin factor).  With a fixed budget of HSC solves, the trapezoid rule is most
accurate when points are dense where n(E) curves.  The surrogate (an FP32 network trained on
the solver's own outputs) predicts, for a device described by (E, disorder sigma, Nx, Ny),
log D(E) (D = DOS injected by the contacts) and log T(E); from it

    g(E)   = D(E) (f_L(E) + f_R(E)) / 2           (the predicted integrand)
    rho(E) ~ |g''(E)|^(1/3) + floor                (point density minimising the trapezoid error)

and the chosen energies are the candidates at equal steps of the cumulative density.  The HSC
solve stays the arbiter: the integrand is computed by the solver at every chosen energy, the
trapezoid error of each interval is estimated from divided differences of the solved values,
and the worst intervals get extra solves (bounded budget).

Everything numerical runs in the library (solves, totals, network training and inference);
this module holds the host logic: features, initialisation, the proposal and the quadrature.
"""
from __future__ import annotations

import numpy as np

from .hsc import HSC_DIAG_GL, HSC_SPECTRAL_LR, HSC_TRANS, Context, solve, totals
from .mlp import MLP

WIDTHS = (4, 256, 256, 2)
LOG_FLOOR = 1e-12


def features(E, sigma, nx, ny):
    """Network inputs [n, 4] (float32): E / 6, sigma / 0.5, (Nx - 28) / 8, (Ny - 28) / 8."""
    E = np.asarray(E, dtype=np.float64).ravel()
    out = np.empty((E.size, 4), np.float32)
    out[:, 0] = E / 6.0
    out[:, 1] = sigma / 0.5
    out[:, 2] = (nx - 28.0) / 8.0
    out[:, 3] = (ny - 28.0) / 8.0
    return out


def observables(ctx: Context, tree, n_sites, energies, eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, batch=0):
    """Solve and reduce: per energy the contact-injected DOS D, the electron density n and T (numpy)."""
    out = solve(ctx, tree, energies, eta=eta, kT=kT, mu_L=mu_L, mu_R=mu_R,
                want=HSC_DIAG_GL | HSC_TRANS | HSC_SPECTRAL_LR, batch=batch, precision=0)
    tt = totals(ctx, out, n_sites).cpu().numpy()
    return {"D": tt[:, 2], "n": tt[:, 1], "T": out["trans"].cpu().numpy(), "status": out["status"].cpu().numpy()}


def targets(D, T, n_sites):
    """[log(D / n_sites), log(T)], both floored at 1e-12."""
    return np.stack([np.log(np.maximum(np.asarray(D) / n_sites, LOG_FLOOR)),
                     np.log(np.maximum(np.asarray(T), LOG_FLOOR))], axis=1)


def xavier_init(widths, seed):
    """Flat parameters: W ~ U(-a, a), a = sqrt(6 / (fan_in + fan_out)); b = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(widths[:-1], widths[1:]):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


class Surrogate:
    """Trained network plus the target standardisation."""

    def __init__(self, ctx: Context, seed=0, widths=WIDTHS):
        self.net = MLP(ctx, widths)
        self.net.set_params(xavier_init(widths, seed))
        self.mean = np.zeros(widths[-1])
        self.std = np.ones(widths[-1])
        self.seed = seed

    def fit(self, X, Y, epochs=300, batch=200, lr=1e-3):
        """Adam on standardised targets, shuffled mini-batches; returns the per-step losses."""
        Y = np.asarray(Y, dtype=np.float64)
        self.mean = Y.mean(axis=0)
        self.std = np.where(Y.std(axis=0) > 0, Y.std(axis=0), 1.0)
        Ys = ((Y - self.mean) / self.std).astype(np.float32)
        n = len(X)
        batch = min(batch, n)
        per = n // batch
        rng = np.random.default_rng(self.seed + 1)
        order = np.concatenate([rng.permutation(n)[:per * batch] for _ in range(epochs)]).astype(np.int32)
        return self.net.train(X, Ys, steps=epochs * per, lr=lr, batch=batch, order=order)

    def predict(self, X):
        """Un-standardised outputs [n, 2]: (log(D / n_sites), log T)."""
        y = self.net.forward(X).cpu().numpy().astype(np.float64)
        return y * self.std + self.mean


def fermi(E, mu, kT):
    x = (np.asarray(E, dtype=np.float64) - mu) / kT
    return np.where(x > 0, np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))), 1.0 / (1.0 + np.exp(-np.abs(x))))


def proposal(cand, g, K, floor=1.0, rel_support=1e-6):
    """K sorted candidate indices (both ends included) at equal steps of the cumulative point
    density rho = |g''|^(1/3) + floor * mean(|g''|^(1/3)) * [g > rel_support * max g] over the
    candidate grid: curvature-driven points plus an even share wherever the predicted integrand
    is not negligible."""
    cand = np.asarray(cand, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    M = cand.size
    if K >= M:
        return np.arange(M)
    d2 = np.zeros(M)
    h0, h1 = np.diff(cand)[:-1], np.diff(cand)[1:]
    d2[1:-1] = 2.0 * ((g[2:] - g[1:-1]) / h1 - (g[1:-1] - g[:-2]) / h0) / (h0 + h1)
    d2[0], d2[-1] = d2[1], d2[-2]
    rho = np.abs(d2) ** (1.0 / 3.0)
    base = rho.mean()
    if not base > 0:
        rho = np.ones(M)
    else:
        rho = rho + floor * base * (g > rel_support * g.max())
        rho = np.maximum(rho, 1e-3 * base)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(cand))])
    idx = np.unique(np.clip(np.searchsorted(cdf, np.linspace(0.0, cdf[-1], K)), 0, M - 1))
    idx = np.union1d(idx, [0, M - 1])
    # fill up to K: split the interval with the largest density mass that still has room
    while idx.size < K:
        mass = cdf[idx[1:]] - cdf[idx[:-1]]
        mass[np.diff(idx) < 2] = -1.0
        j = int(np.argmax(mass))
        if mass[j] < 0:
            break
        idx = np.union1d(idx, [(idx[j] + idx[j + 1]) // 2])
    while idx.size > K:   # drop the interior point whose neighbours are closest in density mass
        gap = cdf[idx[2:]] - cdf[idx[:-2]]
        idx = np.delete(idx, 1 + int(np.argmin(gap)))
    return idx


def trapezoid(E, f):
    E = np.asarray(E, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    return float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(E)))


def interval_errors(E, f):
    """Estimated trapezoid error per interval: h^3 |f''| / 12 with f'' from the second divided
    difference of the neighbouring triples (the larger of the two)."""
    E = np.asarray(E, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    h = np.diff(E)
    if E.size < 3:
        return np.zeros(h.size)
    dd = 2.0 * ((f[2:] - f[1:-1]) / h[1:] - (f[1:-1] - f[:-2]) / h[:-1]) / (h[1:] + h[:-1])
    left = np.concatenate([[0.0], np.abs(dd)])    # triple ending at the interval's right point
    right = np.concatenate([np.abs(dd), [0.0]])   # triple starting at the interval's left point
    return h ** 3 * np.maximum(left, right) / 12.0


class Integrator:
    """Charge of one device by the trapezoid rule on a subset of the candidate energies.

    The support is the open lead band (lo, hi): the contacts inject electrons only there, and at
    its edges the lead broadening vanishes.  A grid is integrated over its candidates inside the
    support plus the first and last candidate inside it; every integrand value is an HSC
    result (cached and counted)."""

    def __init__(self, ctx, tree, n_sites, cand, support, kT=0.025, mu_L=0.1, mu_R=-0.1, eta=1e-8):
        self.ctx, self.tree, self.n_sites = ctx, tree, n_sites
        self.cand = np.asarray(cand, dtype=np.float64)
        self.inside_mask = (self.cand > support[0]) & (self.cand < support[1])
        self.inside = np.flatnonzero(self.inside_mask)
        if self.inside.size < 2:
            raise ValueError("fewer than two candidates inside the support")
        self.kw = dict(eta=eta, kT=kT, mu_L=mu_L, mu_R=mu_R)
        self.val = {}
        self.solves = 0

    def grid(self, idx):
        idx = np.asarray(idx, dtype=np.int64)
        idx = idx[self.inside_mask[idx]]
        return np.union1d(idx, [self.inside[0], self.inside[-1]])

    def need(self, idx):
        new = sorted(int(i) for i in self.grid(idx) if int(i) not in self.val)
        for s in range(0, len(new), 512):
            chunk = new[s:s + 512]
            ob = observables(self.ctx, self.tree, self.n_sites, self.cand[chunk], **self.kw)
            if (ob["status"] != 0).any():
                raise RuntimeError(f"solver status {ob['status'][ob['status'] != 0][:4]} on the charge grid")
            for i, v in zip(chunk, ob["n"]):
                self.val[i] = float(v)
            self.solves += len(chunk)

    def values(self, idx):
        g = self.grid(idx)
        self.need(g)
        return g, np.array([self.val[int(i)] for i in g])

    def charge(self, idx):
        g, v = self.values(idx)
        return trapezoid(self.cand[g], v)

    def cost(self, idx):
        """Solves a grid needs."""
        return int(self.grid(idx).size)

    def refine(self, idx, tol, budget, per_round=16):
        """Add solves where the estimated interval error exceeds tol / (number of points), worst
        first, at most `budget` of them."""
        idx = self.grid(idx)
        K = idx.size
        added = 0
        while added < budget:
            idx, v = self.values(idx)
            err = interval_errors(self.cand[idx], v)
            new = []
            for j in np.argsort(-err):
                if err[j] <= tol / K or len(new) >= min(per_round, budget - added):
                    break
                a, b = idx[j], idx[j + 1]
                if b - a >= 2:
                    new.append((a + b) // 2)
            if not new:
                break
            idx = np.union1d(idx, new)
            added += len(new)
        return idx, added


def dataset(ctx, items, n_energies, seed, e_range=(-6.0, 6.0)):
    """Training samples from the solver: per device (dict with tree, n_sites, sigma, nx, ny)
    n_energies energies drawn uniformly in e_range."""
    rng = np.random.default_rng(seed)
    X, Y = [], []
    for it in items:
        E = np.sort(rng.uniform(e_range[0], e_range[1], n_energies))
        ob = observables(ctx, it["tree"], it["n_sites"], E)
        X.append(features(E, it["sigma"], it["nx"], it["ny"]))
        Y.append(targets(ob["D"], ob["T"], it["n_sites"]))
    return np.concatenate(X), np.concatenate(Y)


def predicted_integrand(surrogate, item, cand, kT=0.025, mu_L=0.1, mu_R=-0.1):
    """g(E) = D(E) (f_L + f_R) / 2 from the surrogate's log D prediction."""
    pred = surrogate.predict(features(cand, item["sigma"], item["nx"], item["ny"]))
    return np.exp(pred[:, 0]) * item["n_sites"] * 0.5 * (fermi(cand, mu_L, kT) + fermi(cand, mu_R, kT))


def equal_cost(ctx, surrogate, item, cand, support, totals_, refine_frac=0.25, tol_rel=1e-4, kT=0.025, mu_L=0.1,
               mu_R=-0.1, floor=1.0):
    """Charge errors at equal numbers S of in-support solves (S in totals_), every grid judged by
    the solver:
      guided          S (1 - refine_frac) points from the surrogate's proposal, then the worst
                      intervals of the solved values split until S solves are spent;
      uniform_refined the same refinement from S (1 - refine_frac) evenly spaced points (the method
                      without the network);
      uniform         S evenly spaced points in the support (the plain grid).
    Returns the per-S errors and, per method, the fewest solves among totals_ that reach tol_rel."""
    cand = np.asarray(cand, dtype=np.float64)
    integ = Integrator(ctx, item["tree"], item["n_sites"], cand, support, kT=kT, mu_L=mu_L, mu_R=mu_R)
    inside = integ.inside
    q_dense = integ.charge(inside)
    g = predicted_integrand(surrogate, item, cand[inside], kT, mu_L, mu_R)

    def uniform_in(k):
        return inside[np.unique(np.round(np.linspace(0, inside.size - 1, k)).astype(int))]

    def err(idx):
        return abs(integ.charge(idx) - q_dense) / abs(q_dense)

    rows = []
    for S in totals_:
        if S >= inside.size:
            continue
        K0 = max(3, int(round(S * (1.0 - refine_frac))))
        gi = inside[proposal(cand[inside], g, K0, floor=floor)]
        gi, _ = integ.refine(gi, 0.0, S - integ.cost(gi))
        ui = uniform_in(K0)
        ui, _ = integ.refine(ui, 0.0, S - integ.cost(ui))
        un = uniform_in(S)
        rows.append({"solves": S, "guided": err(gi), "guided_solves": integ.cost(gi),
                     "uniform_refined": err(ui), "uniform_refined_solves": integ.cost(ui),
                     "uniform": err(un), "uniform_solves": integ.cost(un)})

    def first(key):
        ok = [r["solves"] for r in rows if r[key] <= tol_rel]
        return min(ok) if ok else None

    def stays(key):
        # fewest solves from which every larger budget of the sweep stays within tol_rel (the
        # error of a grid over a spiky integrand is not monotone in its size)
        s = None
        for r in reversed(rows):
            if r[key] > tol_rel:
                break
            s = r["solves"]
        return s

    keys = ("guided", "uniform_refined", "uniform")
    return {"dense_solves": int(inside.size), "rows": rows, "tol_rel": tol_rel,
            "solves_to_tol": {k: stays(k) for k in keys}, "first_within_tol": {k: first(k) for k in keys}}


def study(ctx, surrogate, item, cand, K, support, budget=64, tol_rel=1e-4, kT=0.025, mu_L=0.1, mu_R=-0.1,
          sweep=(16, 24, 32, 48, 64, 96, 128, 256)):
    """Charge of one device on several grids of the candidate energies, all judged by the solver:
    dense (every candidate in the support), guided (K proposed from the surrogate's integrand,
    then refined within `budget` extra solves), uniform (every (len(cand) // K)-th candidate, the
    plain grid of the same size) and uniform_in_support (K evenly spaced candidates of the
    support).  `sweep` reports, for smaller K, the guided proposal against uniform_in_support."""
    cand = np.asarray(cand, dtype=np.float64)
    integ = Integrator(ctx, item["tree"], item["n_sites"], cand, support, kT=kT, mu_L=mu_L, mu_R=mu_R)
    inside = integ.inside
    q_dense = integ.charge(inside)
    g = predicted_integrand(surrogate, item, cand[inside], kT, mu_L, mu_R)

    def guided(k):
        return inside[proposal(cand[inside], g, k)]

    def uniform_in(k):
        return inside[np.unique(np.round(np.linspace(0, inside.size - 1, k)).astype(int))]

    def entry(grid):
        q = integ.charge(grid)
        return {"charge": q, "rel_err": abs(q - q_dense) / abs(q_dense), "solves": integ.cost(grid)}

    idx0 = guided(K)
    res = {"dense": entry(inside), "guided_proposal": entry(idx0)}
    idx, added = integ.refine(idx0, tol_rel * abs(res["guided_proposal"]["charge"]), budget)
    res["guided"] = entry(idx)
    res["refine_added"] = int(added)
    res["uniform"] = entry(np.arange(0, cand.size, max(cand.size // K, 1)))
    res["uniform_in_support"] = entry(uniform_in(K))
    res["sweep"] = [{"K": k, "guided": entry(guided(k))["rel_err"],
                     "uniform_in_support": entry(uniform_in(k))["rel_err"]}
                    for k in sweep if k < inside.size]
    res["solves_total"] = integ.solves
    return res
