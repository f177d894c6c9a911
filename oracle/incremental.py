"""Large-instance renderings of O1 (OMP) and O2 (CLOMP) in float64.

Test infrastructure only (see the package docstring).

The plain oracles in omp.py and clomp.py recompute everything from the
definitions at every step: OMP solves the least squares on the support from
scratch by Householder QR at every iteration (the OMP row of the table of
s-forward blocks), and CLOMP forms A_S s and A_S^T u on the gathered columns for
every Adam step.  At the largest workloads (a flattened 256 x 256 image: n =
65536, m = 19661, k = 2048) that is days of CPU time.  The two functions here
compute the same quantities through identities that hold exactly in real
arithmetic, with nothing else changed (same selection rule, same Adam
definition, same order of operations per iteration):

  omp_cgs2_fp64    the least squares on the growing support by an updated QR
                   factorisation A_S = Q R: each new column is orthogonalised
                   against Q by classical Gram-Schmidt applied twice (the
                   standard re-orthogonalisation that keeps Q orthonormal to
                   working precision), z = Q^T y grows by one entry, the
                   residual of the least squares is y - Q z and x_S solves
                   R x_S = z.
  clomp_gram_fp64  the coefficient-fit gradient mask * A^T (A (mask*s) - y)
                   restricted to the support is A_S^T A_S s_S - A_S^T y =
                   G_S s_S - b_S; G_S and b_S grow by one row and column per
                   selected atom.  Off-support coordinates of s and of the Adam
                   moments stay exactly zero in the plain rendering (their
                   gradient is zero and their moments start at zero), so only
                   the support vector is carried.

Both take A as an (m, n) array and work fastest when A is the transposed view
of a C-contiguous (n, m) float64 array (atom-major storage), since the
correlation A^T r then reads rows.  They are pinned against the plain
oracles (same supports, coefficients to rounding) in the CPU test suite.
"""

import numpy as np
import scipy.linalg

from .grad import adam_step_fp64
from .lstsq import lstsq_support
from .omp import SolveResult, argmax_unselected, ST_NAN, ST_K_CAPPED, ST_ZERO_Y


def _atom_major(A):
    """(m, n) float64 view of A and its (n, m) transpose (a view when A is
    itself the transpose of an atom-major float64 array)."""
    A = np.asarray(A, dtype=np.float64)
    return A, A.T


def omp_cgs2_fp64(A, y, k, A_refine=None):
    """Plain OMP (selection by max |A^T r|, least squares on the support) with
    an updated QR factorisation.  A_refine: matrix for the final least squares
    and residual norm (default A); the selection always runs on A."""
    A, At = _atom_major(A)
    y = np.asarray(y, dtype=np.float64)
    m, n = A.shape
    k_eff = min(k, m, n)
    status = ST_K_CAPPED if k > k_eff else 0
    x = np.zeros(n)
    if float(np.linalg.norm(y)) == 0.0:
        return SolveResult([], x, 0.0, [], [], status | ST_ZERO_Y)
    Q = np.zeros((k_eff, m))        # rows: orthonormal basis of span(A_S)
    R = np.zeros((k_eff, k_eff))    # A_S = Q^T R  (Q stored by rows)
    z = np.zeros(k_eff)             # Q y
    S, gaps, hist = [], [], []
    r = y.copy()
    for t in range(k_eff):
        c = At @ r                                   # residual injection
        j, gap, nonfinite = argmax_unselected(c, S)
        if nonfinite:
            status |= ST_NAN
        gaps.append(gap)
        S.append(j)
        q = At[j].copy()
        Qt = Q[:t]
        h1 = Qt @ q                                  # first Gram-Schmidt pass
        q -= Qt.T @ h1
        h2 = Qt @ q                                  # re-orthogonalisation
        q -= Qt.T @ h2
        rho = float(np.linalg.norm(q))
        if not rho > 0.0:
            raise np.linalg.LinAlgError("selected column is dependent on the support")
        R[:t, t] = h1 + h2
        R[t, t] = rho
        Q[t] = q / rho
        z[t] = Q[t] @ y
        r = y - Q[: t + 1].T @ z[: t + 1]            # least-squares residual
        hist.append(float(np.linalg.norm(r)))
    if A_refine is None:
        xS = scipy.linalg.solve_triangular(R, z, lower=False, check_finite=False)
        rn = hist[-1]
    else:
        xS = lstsq_support(A_refine, y, S)
        Ar = np.asarray(A_refine, dtype=np.float64)
        rn = float(np.linalg.norm(y - Ar[:, S] @ xS))
    x[S] = xS
    return SolveResult(S, x, rn, gaps, hist, status)


def clomp_gram_fp64(A, y, k, params, A_refine=None):
    """CLOMP exactly as clomp_fp64 (argmax selection over unselected atoms,
    lr_t = lr_rel |c_j|, eps = eps_rel * sigma, T Adam steps per atom with one
    global step counter, least-squares refinement on A_refine), with the
    gradient on the support formed as G_S s_S - b_S.  No prior."""
    if params.prior_tv != 0.0 or params.resid_tol != 0.0:
        raise ValueError("clomp_gram_fp64 renders the plain loss without early stopping")
    A, At = _atom_major(A)
    Ar = A if A_refine is None else np.asarray(A_refine, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m, n = A.shape
    k_eff = min(k, m, n)
    status = ST_K_CAPPED if k > k_eff else 0
    x = np.zeros(n)
    if float(np.linalg.norm(y)) == 0.0:
        return SolveResult([], x, 0.0, [], [], status | ST_ZERO_Y,
                           {"s_adam": np.zeros(0), "steps": 0, "sigma": 0.0})
    T = params.inner_steps
    AS = np.zeros((k_eff, m))       # rows: the selected columns a_{S_l}
    G = np.zeros((k_eff, k_eff))    # A_S^T A_S
    b = np.zeros(k_eff)             # A_S^T y
    s = np.zeros(k_eff)             # coefficients on the support (selection order)
    mom = np.zeros(k_eff)
    vel = np.zeros(k_eff)
    step = 0
    S, gaps, hist = [], [], []
    eps = sigma = 0.0
    for t in range(k_eff):
        # (i) residual of the current estimate
        r = y - AS[:t].T @ s[:t]
        if t > 0:
            hist.append(float(np.linalg.norm(r)))
        # (ii) residual injection and argmax selection
        c = At @ r
        j, gap, nonfinite = argmax_unselected(c, S)
        if t == 0:
            sigma = float(np.max(np.abs(c)))
            eps = params.eps_rel * sigma
        lr = params.lr_rel * float(abs(c[j]))
        if nonfinite:
            status |= ST_NAN
        gaps.append(gap)
        # (iii) mask update; the Gram matrix and b grow by the new atom
        S.append(j)
        AS[t] = At[j]
        g_new = AS[: t + 1] @ At[j]
        G[t, : t + 1] = g_new
        G[: t + 1, t] = g_new
        b[t] = At[j] @ y
        # (iv) T Adam steps on the support coefficients
        Gt, bt = G[: t + 1, : t + 1], b[: t + 1]
        st, mt, vt = s[: t + 1], mom[: t + 1], vel[: t + 1]
        for _ in range(T):
            step += 1
            g = Gt @ st - bt
            st, mt, vt = adam_step_fp64(st, g, mt, vt, step, lr, params.beta1,
                                        params.beta2, eps)
        s[: t + 1], mom[: t + 1], vel[: t + 1] = st, mt, vt
    r = y - AS.T @ s
    hist.append(float(np.linalg.norm(r)))
    s_adam = s.copy()
    xS = lstsq_support(Ar, y, S)
    x[S] = xS
    rn = float(np.linalg.norm(y - Ar[:, S] @ xS))
    return SolveResult(S, x, rn, gaps, hist, status,
                       {"s_adam": s_adam, "steps": step, "sigma": sigma})
