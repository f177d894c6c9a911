"""O3 exhaustive support search (tiny instances only).

Test infrastructure only (see the package docstring).

The sparse reconstruction problem of Eq. (2) asks for the fewest non-zeros that
fit y.  For a fixed sparsity k its exact solution is the support of size k with
the smallest least-squares residual, found here by trying every subset.  Used
to pin OMP and CLOMP on n <= 16, k <= 3.
"""

import itertools

import numpy as np

from .lstsq import lstsq_support


def bruteforce_support(A, y, k):
    """Return (best_support_sorted, best_resid_norm, all_resids_dict)."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m, n = A.shape
    if n > 16 or k > 3:
        raise ValueError("brute force is limited to n <= 16, k <= 3")
    best, best_r, table = None, np.inf, {}
    for S in itertools.combinations(range(n), k):
        xS = lstsq_support(A, y, S)
        rn = float(np.linalg.norm(y - A[:, list(S)] @ xS))
        table[S] = rn
        if rn < best_r:
            best, best_r = list(S), rn
    return best, best_r, table
