"""F1 paper-mode CLOMP (multi-atom selection) in float64.

Test infrastructure only (see the package docstring).

The experiments run CLOMP with a normalised cut-off threshold T_h for the
support selected in each iteration and a maximum number of iterations R
(T_h = 0.7, R = 200 unless stated otherwise; Results, synthetic 1-D data).
The CLOMP section describes the multi-position selection ("identifies
multiple positions in a single iteration"): |A^T r| is normalised by an
activation f, cut by the unit step of the CLOMP figure, and OR-ed into the
mask; then s is learned by back-propagation.

One iteration it = 0 .. R-1 of this oracle:
  (i)   r = y - A (mask * s)
  (ii)  c = A^T r;  cmax = max_j |c_j| over all columns
  (iii) new = { j not in mask : |c_j| >= T_h * cmax }; the mask takes them
        when the support stays within k_eff = min(k, m, n), otherwise the
        whole batch is refused and the K-capped status bit is set
  (iv)  one Adam step on the masked coefficients:
        g = mask * A^T (A (mask * s) - y) = -(mask * c)
After the R iterations the coefficients are refined by least squares on the
support (increasing index order) and the FP64 residual norm is reported.

Readings fixed here (the paper leaves them open):
  * f(c) = |c| / max|c| over all columns, selected ones included, and a
    column is new when f >= T_h (the figure's unit step, read as selecting
    where the normalised score reaches the threshold);
  * one Adam step per iteration (beta1 = 0.9, beta2 = 0.999, one step counter,
    zero initial state); lr at iteration it = lr_rel * cmax_it, eps =
    eps_rel * sigma with sigma = cmax at it = 0 (the hot path's scale
    reading with the normaliser in place of the selected correlation);
  * the loop stops early when ||r|| <= resid_tol * ||y|| (Eq. (2)'s epsilon,
    which the paper does not value; 0 disables it) or when cmax is 0;
    non-finite correlations set the NaN bit and stop the loop;
  * a batch of new columns that would exceed k_eff is refused whole (no
    ordering among the batch is implied by the method), so the support is
    the union of the accepted batches.
"""

from dataclasses import dataclass

import numpy as np

from .grad import adam_step_fp64
from .lstsq import lstsq_support
from .omp import SolveResult, ST_NAN, ST_K_CAPPED, ST_ZERO_Y, ST_EARLY_STOP


@dataclass(frozen=True)
class PaperParams:
    threshold: float = 0.7     # T_h
    max_iters: int = 200       # R
    lr_rel: float = 0.05
    beta1: float = 0.9
    beta2: float = 0.999
    eps_rel: float = 1e-8
    resid_tol: float = 0.0     # stop when ||r|| <= resid_tol * ||y|| (Eq. (2)'s epsilon)


def clomp_paper_fp64(A, y, k, params=PaperParams(), A_refine=None):
    """Paper-mode CLOMP on one signal.  Returns SolveResult with the support in
    increasing index order, gaps = per-iteration relative distance of the
    nearest unselected score to the threshold, and extra = {'s_adam': s on
    the support before refinement, 'iters': iterations run, 'sigma',
    'batches': the accepted batches (sorted lists) in order}."""
    A = np.asarray(A, dtype=np.float64)
    Ar = A if A_refine is None else np.asarray(A_refine, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m, n = A.shape
    k_eff = min(k, m, n)
    status = ST_K_CAPPED if k > k_eff else 0
    x = np.zeros(n)
    empty = {"s_adam": np.zeros(0), "iters": 0, "sigma": 0.0, "batches": []}
    ynorm = float(np.linalg.norm(y))
    if ynorm == 0.0:
        return SolveResult([], x, 0.0, [], [], status | ST_ZERO_Y, empty)

    s = np.zeros(n)
    mom = np.zeros(n)
    vel = np.zeros(n)
    mask = np.zeros(n, dtype=bool)
    sigma = eps = 0.0
    gaps, hist, batches = [], [], []
    it = 0
    for it in range(params.max_iters):
        r = y - A @ np.where(mask, s, 0.0)
        hist.append(float(np.linalg.norm(r)))
        if params.resid_tol > 0.0 and hist[-1] <= params.resid_tol * ynorm:
            status |= ST_EARLY_STOP
            break
        c = A.T @ r
        score = np.abs(c)
        if not np.all(np.isfinite(score)):
            status |= ST_NAN
            break
        cmax = float(score.max())
        if cmax == 0.0:
            break
        if it == 0:
            sigma = cmax
            eps = params.eps_rel * sigma
        f = score / cmax
        thr = params.threshold
        new = np.flatnonzero((~mask) & (f >= thr))
        free = f[~mask]
        gaps.append(float(np.min(np.abs(free - thr)) / thr) if free.size else 1.0)
        if new.size:
            if int(mask.sum()) + new.size <= k_eff:
                mask[new] = True
                batches.append(new.tolist())
            else:
                status |= ST_K_CAPPED
        g = np.where(mask, -c, 0.0)
        s, mom, vel = adam_step_fp64(s, g, mom, vel, it + 1, params.lr_rel * cmax,
                                     params.beta1, params.beta2, eps)
    S = np.flatnonzero(mask).tolist()
    s_adam = s[S].copy()
    xS = lstsq_support(Ar, y, S) if S else np.zeros(0)
    x[S] = xS
    rn = float(np.linalg.norm(y - Ar[:, S] @ xS)) if S else float(np.linalg.norm(y))
    return SolveResult(S, x, rn, gaps, hist, status,
                       {"s_adam": s_adam, "iters": it + 1, "sigma": sigma,
                        "batches": batches})
