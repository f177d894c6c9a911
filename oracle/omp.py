"""O1 plain orthogonal matching pursuit in float64.

Test infrastructure only (see the package docstring).

OMP as the paper describes its parent algorithm (Methods, "Coefficients
learning on OMP (CLOMP)", and the OMP panel of the CLOMP figure): each iteration
correlates the residual with every column of A (A^T r), takes the column of
maximum absolute correlation ("basic OMP only identifies the maximum"), adds it
to the support, recomputes the coefficients on the support by least squares
(the OMP row of the s-forward table: pinv(A(:, Mask)) applied to y), and forms
the new residual.  The loop runs k_eff = min(k, m, n) times (the l0 budget of
Eq. (2) given as k); an optional relative residual tolerance stands in for the
epsilon of Eq. (2), which the paper never values.

Readings fixed here (the paper is silent):
  * ties in |A^T r| go to the lowest column index;
  * already-selected columns are excluded from the argmax (in exact arithmetic
    their correlation is zero anyway);
  * y == 0 returns the empty support and x = 0 with the ZERO_Y flag.
"""

from dataclasses import dataclass, field

import numpy as np

from .lstsq import lstsq_support

# Per-instance status flags of the oracle (meanings mirror the GPU library's).
ST_NAN = 1            # a non-finite value reached the selection
ST_K_CAPPED = 2       # k was larger than min(m, n)
ST_ZERO_Y = 4         # y == 0: nothing to select
ST_EARLY_STOP = 16    # residual tolerance reached before k_eff atoms


@dataclass
class SolveResult:
    support: list                 # selected columns in selection order
    x: np.ndarray                 # length n, zeros off the support
    resid_norm: float             # ||y - A_S x_S||_2 (float64)
    gaps: list                    # per iteration (|c|_(1) - |c|_(2)) / |c|_(1)
    resid_hist: list              # ||r_t|| after each iteration
    status: int = 0
    extra: dict = field(default_factory=dict)


def selection_gap(score):
    """Relative gap between the largest and second-largest finite scores."""
    fin = score[np.isfinite(score)]
    if fin.size < 2:
        return 1.0
    top2 = np.partition(fin, fin.size - 2)[-2:]
    hi, lo = float(top2[1]), float(top2[0])
    return 0.0 if hi <= 0.0 else (hi - lo) / hi


def argmax_unselected(c, selected):
    """Index of max |c| over columns not yet selected; lowest index on ties.

    Returns (j, gap, nonfinite).  np.argmax returns the first occurrence of the
    maximum, which is the lowest-index tie-break.
    """
    score = np.abs(c)
    nonfinite = not np.all(np.isfinite(score))
    score = np.where(np.isnan(score), np.inf, score)
    score[list(selected)] = -np.inf
    j = int(np.argmax(score))
    return j, selection_gap(score), nonfinite


def omp_fp64(A, y, k, resid_tol=0.0):
    """Plain OMP.  A: (m, n), y: (m,), k: requested sparsity."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m, n = A.shape
    k_eff = min(k, m, n)
    status = ST_K_CAPPED if k > k_eff else 0
    x = np.zeros(n)
    ynorm = float(np.linalg.norm(y))
    if ynorm == 0.0:
        return SolveResult([], x, 0.0, [], [], status | ST_ZERO_Y)

    S, gaps, hist = [], [], []
    r = y.copy()
    xS = np.zeros(0)
    for _ in range(k_eff):
        c = A.T @ r                                  # residual injection
        j, gap, nonfinite = argmax_unselected(c, S)
        if nonfinite:
            status |= ST_NAN
        gaps.append(gap)
        S.append(j)                                  # mask update
        xS = lstsq_support(A, y, S)                  # s forward: pinv(A_S) y
        r = y - A[:, S] @ xS
        hist.append(float(np.linalg.norm(r)))
        if resid_tol > 0.0 and hist[-1] <= resid_tol * ynorm:
            if len(S) < k_eff:
                status |= ST_EARLY_STOP
            break
    x[S] = xS
    return SolveResult(S, x, float(np.linalg.norm(r)), gaps, hist, status)
