"""F2 total-variation prior (Methods, Eq. (4) and Eq. (5)) in float64.

Test infrastructure only (see the package docstring).

The reconstruction model of Eq. (4) adds weighted prior terms to the residual
loss; Eq. (5) gives the total variation of a 1-D signal x of length n as the
sum of the squared differences of neighbouring samples divided by n.  The
signal is x = D s with D the DCT basis (Results, synthetic data: the DCT
matrix is chosen as D).  With the prior, CLOMP's loss on its mask is

    L(s) = 1/2 ||y - A (mask*s)||^2 + w * TV(D (mask*s))

whose gradient is

    g = mask * ( A^T (A (mask*s) - y) + w * (2/n) D^T Delta^T Delta D (mask*s) )

with Delta the (n-1) x n forward-difference matrix.  The refinement
minimises the same loss over the support:
argmin_x 1/2 ||y - A_S x||^2 + w TV(D_S x), the least-squares problem of
the stacked matrix [A_S ; sqrt(2w/n) Delta D_S] against [y ; 0].

Readings: D is the orthonormal DCT-II synthesis matrix (column k is the k-th
DCT-II basis vector, so atom k of A = M D carries frequency k); the prior
acts on the masked coefficients (the signal the masked layer reconstructs);
w is a free weight (the paper sets prior weights empirically and gives no
value).  Everything here forms D and Delta explicitly.
"""

import numpy as np
import scipy.linalg


def dct_synthesis(n):
    """Orthonormal DCT-II synthesis matrix: D[j, k] = c_k cos(pi k (2j+1) / (2n)),
    c_0 = sqrt(1/n), c_k = sqrt(2/n) for k > 0."""
    j = np.arange(n, dtype=np.float64)[:, None]
    k = np.arange(n, dtype=np.float64)[None, :]
    D = np.cos(np.pi * k * (2.0 * j + 1.0) / (2.0 * n)) * np.sqrt(2.0 / n)
    D[:, 0] = np.sqrt(1.0 / n)
    return D


def forward_difference(n):
    """(n-1) x n matrix with (Delta x)_j = x_j - x_{j+1}."""
    Dl = np.zeros((max(n - 1, 0), n))
    idx = np.arange(n - 1)
    Dl[idx, idx] = 1.0
    Dl[idx, idx + 1] = -1.0
    return Dl


def tv_1d(x):
    """Eq. (5): (1/n) * sum_{j=1}^{n-1} (x_j - x_{j+1})^2."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    return float(np.sum((x[:-1] - x[1:]) ** 2) / n)


def tv_grad_coeffs(s_masked, D):
    """Gradient of TV(D s) with respect to s, at s = s_masked:
    (2/n) D^T Delta^T Delta D s."""
    n = D.shape[0]
    Dl = forward_difference(n)
    x = D @ s_masked
    return (2.0 / n) * (D.T @ (Dl.T @ (Dl @ x)))


def lstsq_support_tv(A, y, S, w, D):
    """argmin_x 1/2 ||y - A[:, S] x||^2 + w * TV(D[:, S] x) by Householder QR of
    the stacked matrix [A_S ; sqrt(2w/n) Delta D_S]."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    S = list(S)
    if not S:
        return np.zeros(0)
    n = D.shape[0]
    Dl = forward_difference(n)
    top = A[:, S]
    bottom = np.sqrt(2.0 * w / n) * (Dl @ D[:, S])
    M = np.vstack([top, bottom])
    rhs = np.concatenate([y, np.zeros(bottom.shape[0])])
    Q, R = scipy.linalg.qr(M, mode="economic", check_finite=False)
    return scipy.linalg.solve_triangular(R, Q.T @ rhs, lower=False, check_finite=False)
