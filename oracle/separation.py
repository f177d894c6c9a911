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


def common_prefix(a, b):
    """Number of leading positions where two ordered supports agree."""
    n = 0
    for p, q in zip(a, b):
        if p != q:
            break
        n += 1
    return n


def separated_prefix(base, perturbed, delta):
    """Length of the leading part of base.support that is well separated: the
    selections before the first iteration whose gap is below delta, cut further
    to where every perturbed run still agrees with the base run.  The greedy
    loop is causal, so selections before that point are decided with margin."""
    L = len(base.support)
    for t, g in enumerate(base.gaps):
        if g < delta:
            L = min(L, t)
            break
    for p in perturbed:
        L = min(L, common_prefix(base.support, p.support))
    return L


def perturbed_atoms(At, u, seed, out=None, chunk=4096):
    """At * (1 + u e) with e independent random signs, for an atom-major (n, m)
    array, filled by chunks of atoms (no full-size temporaries).  Returns out."""
    At = np.asarray(At)
    if out is None:
        out = np.empty(At.shape, dtype=np.float64)
    for c, j0 in enumerate(range(0, At.shape[0], chunk)):
        j1 = min(At.shape[0], j0 + chunk)
        e = np.random.default_rng([7, 7, seed, c]).choice([-1.0, 1.0], size=(j1 - j0, At.shape[1]))
        np.multiply(At[j0:j1], 1.0 + u * e, out=out[j0:j1])
    return out


def perturbed_vector(y, u, seed):
    """y * (1 + u e) with e random signs (companion of perturbed_atoms)."""
    y = np.asarray(y, dtype=np.float64)
    return y * (1.0 + u * np.random.default_rng([7, 8, seed]).choice([-1.0, 1.0], size=y.shape))


def separation_report(A, y, k, method="clomp", params=ClompParams(), delta=1e-4, u=2.0 ** -24,
                      seeds=(1, 2), A_refine=None, base=None):
    """(ok, prefix, base): well_separated's verdict and the separated prefix of
    the base support, from the same perturbed runs."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if base is None:
        base = _run(method, A, y, k, params, A_refine)
    pert = []
    for sd in seeds:
        rng = np.random.default_rng([7, 7, sd])
        Ap = A * (1.0 + u * rng.choice([-1.0, 1.0], size=A.shape))
        yp = y * (1.0 + u * rng.choice([-1.0, 1.0], size=y.shape))
        pert.append(_run(method, Ap, yp, k, params, A_refine))
    ok = (not len(base.gaps) or min(base.gaps) >= delta) and all(
        p.support == base.support for p in pert)
    return ok, separated_prefix(base, pert, delta), base
