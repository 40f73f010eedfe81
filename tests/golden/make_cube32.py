"""Write tests/golden/cube32_sampled.json from the CPU oracle only.

The 32^3 cube of the throughput benchmark (t = -1, on-site U[-0.5, 0.5] seed 0,
per-site 1D leads on the x faces, eta = 1e-8, kT = 0.025, mu_L/R = +-0.1).
Eight energies of the 256-point grid linspace(-6, 6, 256) (in and out of the
lead band [-2, 2]) and 64 seeded sites plus the four x-face corner sites:
  gr, gl, a_l, a_r, trans  -- oracle.sampled (refined sparse LU rows of G^r; T from the
                              rows of every left-contact site).
The slab recursive Green's function (oracle.rgf) is not used for T here: like every
unpivoted elimination it loses digits outside the lead band, where T is tiny.
Run:  python tests/golden/make_cube32.py   (one process per energy; about half an hour on 8 cores)
"""
import json
import multiprocessing
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
import oracle  # noqa: E402

E_INDEX = [3, 45, 77, 100, 127, 160, 190, 230]


def _one_energy(args):
    dev, en, sites = args
    return oracle.sampled.solve_sites(dev, [en], 1e-8, 0.025, 0.1, -0.1, sites, want_trans=True)


def main():
    dev = synth.config1_device()
    grid = np.linspace(-6.0, 6.0, 256)
    energies = grid[E_INDEX]
    rng = np.random.default_rng(2024)
    sites = np.unique(np.concatenate([rng.choice(dev.n, 64, replace=False),
                                      [0, 31 * 32 * 32, 31, 32 ** 3 - 1]])).astype(np.int64)
    # one process per energy (each factorisation and its solves run on one core)
    with multiprocessing.get_context("fork").Pool(len(energies)) as pool:
        parts = pool.map(_one_energy, [(dev, float(en), sites) for en in energies])
    s = {k: np.concatenate([p[k] for p in parts]) for k in ("gr", "gl", "a_l", "a_r", "trans")}
    out = {
        "workload": "cube 32^3, t=-1, onsite U[-0.5,0.5] seed 0, eta 1e-8, kT 0.025, mu +-0.1",
        "energy_index": E_INDEX, "energies": energies.tolist(), "sites": sites.tolist(),
        "gr_re": s["gr"].real.tolist(), "gr_im": s["gr"].imag.tolist(),
        "gl_im": s["gl"].imag.tolist(), "gl_re": s["gl"].real.tolist(),
        "a_l": s["a_l"].tolist(), "a_r": s["a_r"].tolist(),
        "trans": s["trans"].tolist(),
    }
    with open(os.path.join(HERE, "cube32_sampled.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
