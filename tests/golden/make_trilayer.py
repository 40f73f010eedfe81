"""Write tests/golden/trilayer_rgf.json from the CPU oracle only.

The graphene / BN / graphene trilayer (116 x 115 sites per layer, 40,020 sites,
in-plane hopping -2.7 eV, BN on-site +-1.4 eV, interlayer 0.4 eV, leads on the
x = 0 edge of layer 0 and the x = Wx-1 edge of layer 2), eta = 1e-8, kT = 0.025,
mu_L/R = +-0.1.  Six energies of the 512-point grid linspace(-3, 3, 512) (all in
the lead band [-5.4, 5.4]); diagonals at 64 seeded sites plus the contact-edge
corners, and T, all from oracle.rgf (slab recursive Green's function along x).
Run:  python tests/golden/make_trilayer.py   (about a minute on 8 cores)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
import oracle  # noqa: E402

E_INDEX = [0, 100, 200, 255, 350, 511]


def main():
    dev = synth.trilayer()
    energies = np.linspace(-3.0, 3.0, 512)[E_INDEX]
    rng = np.random.default_rng(77)
    wx, wy = 116, 115
    corners = [0, wx - 1, wx * (wy - 1), 2 * wx * wy + wx - 1, 3 * wx * wy - 1]
    sites = np.unique(np.concatenate([rng.choice(dev.n, 64, replace=False), corners])).astype(np.int64)
    r = oracle.rgf.solve(dev, energies, 1e-8, 0.025, 0.1, -0.1)
    out = {
        "workload": "trilayer 116x115x3, t=-2.7, BN +-1.4, interlayer 0.4, eta 1e-8, kT 0.025, mu +-0.1",
        "energy_index": E_INDEX, "energies": energies.tolist(), "sites": sites.tolist(),
        "gr_re": r["gr"][:, sites].real.tolist(), "gr_im": r["gr"][:, sites].imag.tolist(),
        "gl_re": r["gl"][:, sites].real.tolist(), "gl_im": r["gl"][:, sites].imag.tolist(),
        "a_l": r["a_l"][:, sites].tolist(), "a_r": r["a_r"][:, sites].tolist(),
        "trans": r["trans"].tolist(),
    }
    with open(os.path.join(HERE, "trilayer_rgf.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
