"""F4 iterative hard thresholding (IHT), the experiments' fast comparison
method, in float64.

Test infrastructure only (see the package docstring).

The table of s-forward blocks gives IHT as s = H_K(s + t A^T r): a gradient
step on 1/2 ||y - A s||^2 followed by the hard threshold H_K that keeps the K
largest magnitudes (its sign implies r = y - A s).  The step t is not valued;
this oracle takes the normalised step of normalised IHT (Blumensath and
Davies): t = ||g_G||^2 / ||A_G g_G||^2 with g = A^T r restricted to the
current support G, which keeps the iteration stable on dictionaries whose
spectral norm exceeds 1 (Gaussian A with n > m).

One iteration it = 0 .. R-1:
  r = y - A s;  g = A^T r
  G = support of s (it > 0), or the K largest |g| (it = 0, where s = 0)
  t = ||g_G||^2 / ||A_G g_G||^2   (0 when the denominator is 0)
  z = s + t g;  s = z on the K largest |z|, 0 elsewhere
(K largest: by magnitude, ties to the lowest index, NaN ranked highest.)
After the R iterations the coefficients are refined by least squares on the
support (increasing index order) and the FP64 residual norm is reported, as
for OMP and CLOMP.

Readings: K = k_eff = min(k, m, n); no backtracking of the normalised step;
R = 200 (the experiments' maximum iteration number) unless given.
"""

import numpy as np

from .lstsq import lstsq_support
from .omp import SolveResult, ST_NAN, ST_K_CAPPED, ST_ZERO_Y


def top_k(z, K):
    """Indices of the K largest |z| (ties: lowest index; NaN highest), and the
    relative gap between the K-th and (K+1)-th magnitudes."""
    a = np.abs(z)
    a = np.where(np.isnan(a), np.inf, a)
    order = np.lexsort((np.arange(a.size), -a))
    sel = np.sort(order[:K])
    if K < a.size and np.isfinite(a[order[K - 1]]) and a[order[K - 1]] > 0:
        gap = float((a[order[K - 1]] - a[order[K]]) / a[order[K - 1]])
    else:
        gap = 1.0
    return sel, gap


def iht_fp64(A, y, k, max_iters=200, A_refine=None):
    """Normalised IHT on one signal.  Returns SolveResult (support in
    increasing index order; gaps = per-iteration relative gap at the top-K
    boundary; extra = {'s_iht': s on the support before refinement,
    'steps': the normalised step of each iteration})."""
    A = np.asarray(A, dtype=np.float64)
    Ar = A if A_refine is None else np.asarray(A_refine, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m, n = A.shape
    K = min(k, m, n)
    status = ST_K_CAPPED if k > K else 0
    x = np.zeros(n)
    if float(np.linalg.norm(y)) == 0.0:
        return SolveResult([], x, 0.0, [], [], status | ST_ZERO_Y,
                           {"s_iht": np.zeros(0), "steps": []})
    s = np.zeros(n)
    G = None
    gaps, hist, steps = [], [], []
    for it in range(max_iters):
        r = y - A @ s
        hist.append(float(np.linalg.norm(r)))
        g = A.T @ r
        if not np.all(np.isfinite(g)):
            status |= ST_NAN
        if G is None:
            G, _ = top_k(g, K)
        gG = g[G]
        den = float(np.sum((A[:, G] @ gG) ** 2))
        t = float(np.sum(gG ** 2)) / den if den > 0.0 else 0.0
        steps.append(t)
        z = s + t * g
        G, gap = top_k(z, K)
        gaps.append(gap)
        s = np.zeros(n)
        s[G] = z[G]
    S = [int(j) for j in G]
    s_iht = s[S].copy()
    xS = lstsq_support(Ar, y, S)
    x[S] = xS
    rn = float(np.linalg.norm(y - Ar[:, S] @ xS))
    return SolveResult(S, x, rn, gaps, hist, status, {"s_iht": s_iht, "steps": steps})
