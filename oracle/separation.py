"""Well-separated instances: when support identity can be asserted.

Test infrastructure only (see the package docstring).

A greedy selection is decided by comparisons of |A^T r|.  When two candidates
are nearly tied, any rounding difference (float32 versus float64, bfloat16
storage, a different summation order) may flip the choice, and every later
iteration then differs.  Support identity between the GPU path and this oracle
is therefore asserted only on instances where
  1. every iteration's relative gap between the best and second-best score
     (paper mode: between the threshold and the nearest unselected score) is
     at least delta, and
  2. the oracle's support is unchanged when every entry of A and y is
     multiplied by (1 + u * e) with e a random sign, for two seeds.
The second condition covers sensitivity of the Adam trajectory, which the
per-iteration gap alone does not see.
"""

import numpy as np

from .clomp import clomp_fp64, ClompParams
from .clomp_paper import clomp_paper_fp64
from .omp import omp_fp64
from .iht import iht_fp64


def _run(method, A, y, k, params, A_refine):
    if method == "omp":
        return omp_fp64(A, y, k, resid_tol=params.resid_tol)
    if method == "iht":
        # gaps: relative gap at the top-K boundary of every iteration
        return iht_fp64(A, y, k, max_iters=getattr(params, "max_iters", 200),
                        A_refine=A_refine)
    if method == "clomp_paper":
        # gaps: distance of the nearest unselected score to the threshold
        return clomp_paper_fp64(A, y, k, params, A_refine=A_refine)
    return clomp_fp64(A, y, k, params, A_refine=A_refine)


def well_separated(A, y, k, method="clomp", params=ClompParams(), delta=1e-4,
                   u=2.0 ** -24, seeds=(1, 2), A_refine=None, base=None):
    """Return (ok, base_result).  `base` may pass a precomputed oracle result."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if base is None:
        base = _run(method, A, y, k, params, A_refine)
    if len(base.gaps) and min(base.gaps) < delta:
        return False, base
    for sd in seeds:
        rng = np.random.default_rng([7, 7, sd])
        Ap = A * (1.0 + u * rng.choice([-1.0, 1.0], size=A.shape))
        yp = y * (1.0 + u * rng.choice([-1.0, 1.0], size=y.shape))
        pert = _run(method, Ap, yp, k, params, A_refine)
        if pert.support != base.support:
            return False, base
    return True, base
