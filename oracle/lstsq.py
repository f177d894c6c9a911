"""O6 least squares on a support, and the FP64 residual-norm check.

Test infrastructure only (see the package docstring).

The OMP row of the paper's table of s-forward blocks (Methods, "The Ultra Small
Model") computes the coefficients on the selected columns with a pseudo-inverse
of A(:, Mask).  The printed entry omits the right-hand side; the reading used
here is s_S = pinv(A_S) y, i.e. the least-squares solution on the support.  It
is computed by Householder QR (LAPACK geqrf through scipy) and a triangular
solve, which is the backward-stable textbook route for a full-column-rank A_S.
"""

import numpy as np
import scipy.linalg


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def lstsq_support(A, y, S):
    """Return x_S = argmin_x ||y - A[:, S] x||_2 (float64, length len(S)).

    A: (m, n) array, y: (m,), S: sequence of distinct column indices.
    An empty support returns an empty vector.
    """
    A = _f64(A)
    y = _f64(y)
    S = list(S)
    if len(S) == 0:
        return np.zeros(0)
    AS = A[:, S]
    Q, R = scipy.linalg.qr(AS, mode="economic", check_finite=False)
    return scipy.linalg.solve_triangular(R, Q.T @ y, lower=False,
                                       check_finite=False)


def resid_norm_fp64(A, y, S, xS):
    """||y - A[:, S] x_S||_2 in float64: the residual of Eq. (2), the quantity
    the reconstruction constraint bounds by epsilon."""
    A = _f64(A)
    y = _f64(y)
    S = list(S)
    if len(S) == 0:
        return float(np.linalg.norm(y))
    r = y - A[:, S] @ _f64(xS)
    return float(np.linalg.norm(r))
