"""O2 coefficients-learning OMP (CLOMP) in float64.

Test infrastructure only (see the package docstring).

CLOMP keeps OMP's residual-injection branch and replaces its least-squares
s-forward block by learnable coefficients (Methods, "General idea of
coefficients learning" and "Coefficients learning on OMP (CLOMP)"):

  residual injection  c = A^T r, scored by |c|; the selected position is OR-ed
                      into a binary Mask (unit-step of the CLOMP figure)
  s forward           s is a vector of n learnable parameters ("structure 1":
                      s itself is the parameter); mask * s goes through a fully
                      connected layer with fixed weights A to give y' = A(mask*s)
  learning            the residual loss is back-propagated into s and an
                      optimiser steps s ("auto-gradient and backpropagation")

One outer iteration t = 0 .. k_eff-1 of this oracle:
  (i)   r = y - A (mask * s)
  (ii)  c = A^T r; j = argmax over unselected columns of |c| (lowest index on ties)
  (iii) mask[j] = 1, S.append(j)
  (iv)  T times: step += 1;  g = mask * A^T (A (mask * s) - y);  Adam(s, g)
After the loop the coefficients are refined by least squares on S (the OMP
s-forward, applied once) and the FP64 residual norm of Eq. (2) is reported.

Readings fixed here (the paper is silent on all of them):
  * selection is the single maximum (the paper's "basic OMP" selection, i.e. a
    normalised cut-off threshold T_h = 1); multi-select with T_h = 0.7 is a
    different mode of the method, not this one;
  * already-selected columns are excluded from the argmax (CLOMP's inexact fit
    leaves their correlations non-zero; excluding them selects exactly k_eff
    distinct atoms);
  * optimiser Adam (beta1 = 0.9, beta2 = 0.999), one global step counter per
    instance, state (s, m, v) starts at zero;
  * the learning rate follows the residual: at iteration t, lr_t = lr_rel *
    |c_j| with c_j the correlation of the atom just selected, and
    eps = eps_rel * sigma with sigma = max_j |a_j^T y| (the first correlation);
    both scale with y, so a power-of-two scaling of y scales every iterate by
    the same power of two.  (A constant lr cannot resolve coefficients several
    decades below the largest one within T steps: Adam's step has the size of
    lr whatever the gradient's magnitude.)
  * loss scale 1/2 ||A(mask*s) - y||^2 (see grad.py).

prior_tv = w > 0 adds the total-variation prior of Eq. (4)-(5) on the signal
D (mask*s) to the loss, in step (iv) and in the refinement (prior.py).

inner='exact' replaces step (iv) by the least-squares s-forward, which turns the
loop into plain OMP (used as a reduction test).

A_refine: matrix used for the final least squares and residual norm.  When the
selection matrix A holds a reduced-precision copy (bfloat16 values), A_refine
holds the float32 master values; by default it is A itself.
"""

from dataclasses import dataclass

import numpy as np

from .grad import adam_step_fp64
from .lstsq import lstsq_support
from .prior import dct_synthesis, lstsq_support_tv, tv_grad_coeffs
from .omp import (SolveResult, argmax_unselected, ST_NAN, ST_K_CAPPED,
                  ST_ZERO_Y, ST_EARLY_STOP)


@dataclass(frozen=True)
class ClompParams:
    inner_steps: int = 32      # T: Adam steps per selected atom
    lr_rel: float = 0.05       # lr_t = lr_rel * |c_j| of the atom selected at t
    beta1: float = 0.9
    beta2: float = 0.999
    eps_rel: float = 1e-8      # eps = eps_rel * sigma
    resid_tol: float = 0.0     # stop when ||r|| <= resid_tol * ||y|| (0: off)
    prior_tv: float = 0.0      # w of the total-variation prior (0: no prior)


def clomp_fp64(A, y, k, params=ClompParams(), inner="adam", A_refine=None):
    """CLOMP on one signal.  Returns SolveResult with extra = {
    's_adam': coefficients on S before refinement (selection order),
    'steps': total Adam steps, 'sigma': max |A^T y|}."""
    A = np.asarray(A, dtype=np.float64)
    Ar = A if A_refine is None else np.asarray(A_refine, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m, n = A.shape
    k_eff = min(k, m, n)
    status = ST_K_CAPPED if k > k_eff else 0
    x = np.zeros(n)
    ynorm = float(np.linalg.norm(y))
    if ynorm == 0.0:
        return SolveResult([], x, 0.0, [], [], status | ST_ZERO_Y,
                           {"s_adam": np.zeros(0), "steps": 0, "sigma": 0.0})

    T = params.inner_steps
    s = np.zeros(n)          # learnable coefficients (all n of them)
    mom = np.zeros(n)        # Adam first moment
    vel = np.zeros(n)        # Adam second moment
    mask = np.zeros(n, dtype=bool)
    step = 0
    S, gaps, hist = [], [], []
    lr = eps = sigma = 0.0
    w_tv = params.prior_tv
    D = dct_synthesis(n) if w_tv > 0.0 else None

    for t in range(k_eff):
        # (i) residual of the current estimate y' = A (mask * s)
        r = y - A @ np.where(mask, s, 0.0)
        if t > 0:
            hist.append(float(np.linalg.norm(r)))
            if params.resid_tol > 0.0 and hist[-1] <= params.resid_tol * ynorm:
                status |= ST_EARLY_STOP
                break
        # (ii) residual injection and argmax selection
        c = A.T @ r
        j, gap, nonfinite = argmax_unselected(c, S)
        if t == 0:
            sigma = float(np.max(np.abs(c)))
            eps = params.eps_rel * sigma
        lr = params.lr_rel * float(abs(c[j]))
        if nonfinite:
            status |= ST_NAN
        gaps.append(gap)
        # (iii) mask update (bitwise OR with the new position)
        mask[j] = True
        S.append(j)
        # (iv) learn s on the mask
        if inner == "exact":
            s[:] = 0.0
            s[S] = lstsq_support(A, y, S)
        else:
            for _ in range(T):
                step += 1
                # g = mask * A^T (A (mask*s) - y); entries off the mask are 0,
                # so only the columns in S are formed.
                AS = A[:, S]
                u = AS @ s[S] - y
                g = np.zeros(n)
                g[S] = AS.T @ u
                if D is not None:
                    g[S] += w_tv * tv_grad_coeffs(np.where(mask, s, 0.0), D)[S]
                s, mom, vel = adam_step_fp64(s, g, mom, vel, step, lr,
                                             params.beta1, params.beta2, eps)

    if not (status & ST_EARLY_STOP):
        r = y - A @ np.where(mask, s, 0.0)
        hist.append(float(np.linalg.norm(r)))
    s_adam = s[S].copy()
    xS = lstsq_support(Ar, y, S) if D is None else lstsq_support_tv(Ar, y, S, w_tv, D)
    x[S] = xS
    rn = float(np.linalg.norm(y - Ar[:, S] @ xS))
    return SolveResult(S, x, rn, gaps, hist, status,
                       {"s_adam": s_adam, "steps": step, "sigma": sigma})
