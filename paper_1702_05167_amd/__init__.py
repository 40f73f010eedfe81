"""MI355X nested-dissection NEGF solver (HSC + HSC-extension, arxiv 1702.05167).

The compute path is libhsc.so (hand-written HIP kernels for gfx950) behind the
C ABI in include/hsc.h; ``hsc`` is its ctypes binding.
"""
from .hsc import (  # noqa: F401
    HSC_DIAG_GR, HSC_DIAG_GL, HSC_TRANS, HSC_SPECTRAL_LR, HSC_BOND_GR, HSC_BOND_GL, Context, Tree, solve, solve_batch, totals, HscError, lib,
    LIB_PATH, poisson_solve, density, scf,
)
from .mlp import MLP  # noqa: F401
from .sweep import sweep  # noqa: F401
