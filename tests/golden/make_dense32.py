"""Write tests/golden/dense32_rgf.json from the CPU oracle only.

The 32^3 cube of the throughput benchmark (t = -1, on-site U[-0.5, 0.5] seed 0,
eta = 1e-8, kT = 0.025, mu_L/R = +-0.1) with whole-face contacts: each x face
couples to a semi-infinite lead continuing the face lattice (on-site 0,
hopping -1, coupling -1), i.e. the dense self-energy blocks of oracle.face.
Four energies of the 256-point grid linspace(-6, 6, 256), all inside the
whole-face lead's band [-6, 6] where T is of order 10-300, and 64 seeded sites
plus the four x-face corner sites:
  gr, gl, a_l, a_r, trans  -- oracle.rgf with dense=True (slab recursion along x,
                              the face blocks on the first and last slab).
The slab recursion is exact up to rounding; it loses relative digits only where
T is tiny (evanescent transport), which none of these energies is.
Run:  python tests/golden/make_dense32.py   (one process per energy; a few minutes on 8 cores)
"""
import json
import multiprocessing
import os
import sys

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "2"

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
import oracle  # noqa: E402

E_INDEX = [45, 100, 127, 190]


def _one_energy(en):
    dev = synth.config1_device()
    return oracle.rgf.solve(dev, [en], 1e-8, 0.025, 0.1, -0.1, dense=True)


def main():
    dev = synth.config1_device()
    grid = np.linspace(-6.0, 6.0, 256)
    energies = grid[E_INDEX]
    rng = np.random.default_rng(2025)
    sites = np.unique(np.concatenate([rng.choice(dev.n, 64, replace=False),
                                      [0, 31 * 32 * 32, 31, 32 ** 3 - 1]])).astype(np.int64)
    with multiprocessing.get_context("fork").Pool(len(energies)) as pool:
        parts = pool.map(_one_energy, [float(en) for en in energies])
    s = {k: np.concatenate([p[k][:, sites] for p in parts]) for k in ("gr", "gl", "a_l", "a_r")}
    out = {
        "workload": "cube 32^3, t=-1, onsite U[-0.5,0.5] seed 0, whole-face leads (eps 0, t_l -1, t_c -1), "
                    "eta 1e-8, kT 0.025, mu +-0.1",
        "energy_index": E_INDEX, "energies": energies.tolist(), "sites": sites.tolist(),
        "gr_re": s["gr"].real.tolist(), "gr_im": s["gr"].imag.tolist(),
        "gl_im": s["gl"].imag.tolist(), "gl_re": s["gl"].real.tolist(),
        "a_l": s["a_l"].tolist(), "a_r": s["a_r"].tolist(),
        "trans": [float(p["trans"][0]) for p in parts],
    }
    with open(os.path.join(HERE, "dense32_rgf.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
