"""CPU oracle for the NEGF diagonals -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct float64 / complex128 reference implementations of
what the GPU hot path computes, written from the paper's definitions:

* Eq. (1): G^r(E) = A(E)^-1 with A = E I - H - Sigma^r.
* Eq. (2): G^<(E) = G^r Sigma^< (G^r)^dagger.

Modules:

* ``negf``    -- lead self-energy (closed-form 1D chain), broadening, Fermi
                 function, and the per-energy quantities built from them.
* ``face``    -- DENSE contact self-energy of a whole face (lead continuing the
                 face lattice), and Sancho-Rubio decimation as its independent check.
* ``dense``   -- the definition itself: dense partial-pivot LU inverse (small n).
* ``rgf``     -- slab-wise recursive Green's function sweeps (Section 2.1), for
                 mid sizes.
* ``sampled`` -- sparse LU (partial pivoting) column solves for sampled sites,
                 usable at any size.
* ``mlp``     -- float64 forward pass, chain-rule gradients and Adam of the
                 surrogate network of the learned energy grid.
* ``scf``     -- the self-consistent NEGF-Poisson loop: 7-point Poisson on the device
                 grid (sparse direct solve), electron density from diag G^<, mixing.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  The GPU path never does: it shares no code with it.
"""
from . import negf, face, dense, rgf, sampled, mlp, scf  # noqa: F401
