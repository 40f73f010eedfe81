"""Write tests/golden/config2_sampled.json from the CPU oracle only.

Four of the 64 uneven cuboids of the batched workload (sides integers in
[16, 48] from default_rng(0), on-site N(0, 0.3^2) from default_rng((0, d)),
t = -1, per-site 1D leads on the x faces, eta = 1e-8, kT = 0.025,
mu_L/R = +-0.1): the smallest (device 14, 16 x 20 x 16), the largest
(device 63, 48 x 43 x 47) and two between them (devices 11 and 5).
Four energies of the 128-point grid linspace(-6, 6, 128): two inside the lead
band (-2, 2), two outside it.  Per device 64 seeded sites plus the two x-face
corners at the origin's row:
  gr, gl, a_l, a_r, trans  -- oracle.sampled (refined sparse-LU rows of G^r; T
                              from the rows of every left-contact site).
Run:  python tests/golden/make_config2.py [processes]   (one process per
(device, energy); the largest device takes most of the time)
"""
import json
import multiprocessing
import os
import sys
import time

# one BLAS thread per worker process (forked workers of a threaded BLAS can spin)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
import oracle  # noqa: E402

DEVICES = [14, 11, 5, 63]
E_INDEX = [20, 50, 70, 115]


def _sites(dev, d):
    rng = np.random.default_rng(7000 + d)
    nx = dev.grid[0]
    extra = [0, nx - 1]
    return np.unique(np.concatenate([rng.choice(dev.n, 64, replace=False), extra])).astype(np.int64)


def _one(args):
    d, en = args
    dev = synth.config2_devices(which=[d])[0]
    t0 = time.time()
    r = oracle.sampled.solve_sites(dev, [en], 1e-8, 0.025, 0.1, -0.1, _sites(dev, d), want_trans=True)
    print(f"device {d} E={en:+.4f}: {time.time() - t0:.0f} s", flush=True)
    return r


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    grid = np.linspace(-6.0, 6.0, 128)
    jobs = [(d, float(grid[k])) for d in DEVICES[::-1] for k in E_INDEX]   # largest device first
    with multiprocessing.get_context("fork").Pool(procs) as pool:
        parts = pool.map(_one, jobs, chunksize=1)
    res = dict(zip(jobs, parts))
    sizes = synth.config2_sizes()
    out = {"workload": "uneven cuboids (sides in [16, 48], seed 0), on-site N(0, 0.3^2), t=-1, eta 1e-8, "
                       "kT 0.025, mu +-0.1, energies linspace(-6, 6, 128)",
           "energy_index": E_INDEX, "energies": grid[E_INDEX].tolist(), "devices": []}
    for d in DEVICES:
        dev = synth.config2_devices(which=[d])[0]
        rows = [res[(d, float(grid[k]))] for k in E_INDEX]
        s = {k: np.concatenate([r[k] for r in rows]) for k in ("gr", "gl", "a_l", "a_r", "trans")}
        out["devices"].append({
            "device": d, "sides": [int(v) for v in sizes[d]], "sites": _sites(dev, d).tolist(),
            "gr_re": s["gr"].real.tolist(), "gr_im": s["gr"].imag.tolist(),
            "gl_im": s["gl"].imag.tolist(), "gl_re": s["gl"].real.tolist(),
            "a_l": s["a_l"].tolist(), "a_r": s["a_r"].tolist(), "trans": s["trans"].tolist()})
    with open(os.path.join(HERE, "config2_sampled.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
