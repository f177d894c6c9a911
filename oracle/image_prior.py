"""F2 image priors (Methods, Eq. (4), Eq. (6), Eq. (7)) and CLOMP on the columns
of one image, in float64.

Test infrastructure only (see the package docstring).

An image X (H x W, here n x a) is reconstructed column by column: column c is
the signal x_c = D s_c with D the DCT basis, and every column is measured with
the same matrix, Y = A S (Eq. (3)).  Eq. (4) adds prior terms to the residual
loss; for images the paper gives

  TV(X) = (1/H) sum_j sum_{i<H-1} (X[i,j] - X[i+1,j])^2
        + (1/W) sum_i sum_{j<W-1} (X[i,j] - X[i,j+1])^2            (Eq. (6))
  LV(X) = (1/B) sum_b std(X_b)                                      (Eq. (7))

with X_b the pixels of block b, a 3 x 3 window sliding with a step smaller
than the window.  The loss of the whole image is

  L(S) = sum_c 1/2 ||y_c - A (mask_c * s_c)||^2 + w_tv TV(X) + w_lv LV(X),
  X = D (Mask * S).

Readings fixed here (the paper states the terms, not these details):
  * D is the orthonormal DCT-II synthesis matrix (prior.dct_synthesis) and the
    priors act on the masked coefficients, as for the 1-D prior;
  * Eq. (6)'s sums run over every pixel pair (its index notation names only
    one index per term); its first term is Eq. (5) applied to every column;
  * LV: every 3 x 3 window lying inside the image, step 1 in both directions,
    B = (H - 2)(W - 2) windows; std is the sample standard deviation (divisor
    8, the default of the deep-learning frameworks the experiments used), and
    its gradient is taken as zero where a window is constant;
  * one weight per term (w_tv for all of Eq. (6), w_lv for Eq. (7)); the paper
    sets them empirically and gives no values;
  * CLOMP on an image (clomp_image_fp64): every outer iteration each column
    selects its own atom from its own residual, then T Adam steps are taken on
    all columns together, each on the loss above (the priors couple
    neighbouring columns); each column keeps its own learning rate
    (lr_rel |c_j| of its selected atom) and eps (eps_rel max_j |a_j^T y_c|),
    the step counter is common;
  * the result is the learned coefficients: LV is not quadratic, so no
    least-squares solve on the support minimises the same loss (the 1-D TV
    refinement of prior.py does, and the image mode does not use it).

The functions compute the priors literally on the pixel image (explicit D,
explicit differences and windows) except where a docstring names an identity.
"""

import numpy as np

from .grad import adam_step_fp64
from .omp import SolveResult, argmax_unselected, ST_NAN, ST_K_CAPPED, ST_ZERO_Y
from .prior import dct_synthesis


def tv_2d(X):
    """Eq. (6) on an H x W image: vertical and horizontal squared differences,
    divided by H and W."""
    X = np.asarray(X, dtype=np.float64)
    H, W = X.shape
    v = np.sum((X[:-1, :] - X[1:, :]) ** 2) / H
    h = np.sum((X[:, :-1] - X[:, 1:]) ** 2) / W
    return float(v + h)


def tv_2d_grad(X):
    """Gradient of Eq. (6) with respect to the pixels."""
    X = np.asarray(X, dtype=np.float64)
    H, W = X.shape
    G = np.zeros_like(X)
    dv = X[:-1, :] - X[1:, :]              # (H-1) x W
    G[:-1, :] += 2.0 * dv / H
    G[1:, :] -= 2.0 * dv / H
    dh = X[:, :-1] - X[:, 1:]              # H x (W-1)
    G[:, :-1] += 2.0 * dh / W
    G[:, 1:] -= 2.0 * dh / W
    return G


LV_WIN = 3      # window side
LV_STEP = 1     # sliding step (smaller than the window)
LV_DDOF = 1     # sample standard deviation


def _windows(H, W):
    """Top-left corners of the 3 x 3 windows inside an H x W image."""
    return [(i, j) for i in range(0, H - LV_WIN + 1, LV_STEP)
            for j in range(0, W - LV_WIN + 1, LV_STEP)]


def lv(X):
    """Eq. (7): mean over the windows of the sample standard deviation."""
    X = np.asarray(X, dtype=np.float64)
    H, W = X.shape
    wins = _windows(H, W)
    if not wins:
        return 0.0
    tot = 0.0
    for i, j in wins:
        tot += float(np.std(X[i:i + LV_WIN, j:j + LV_WIN], ddof=LV_DDOF))
    return tot / len(wins)


def lv_grad(X):
    """Gradient of Eq. (7) with respect to the pixels: each window b adds
    (x_p - mean_b) / ((N - 1) std_b) / B to its N = 9 pixels p (nothing when
    std_b = 0)."""
    X = np.asarray(X, dtype=np.float64)
    H, W = X.shape
    wins = _windows(H, W)
    G = np.zeros_like(X)
    if not wins:
        return G
    N = LV_WIN * LV_WIN
    for i, j in wins:
        blk = X[i:i + LV_WIN, j:j + LV_WIN]
        sd = float(np.std(blk, ddof=LV_DDOF))
        if sd > 0.0:
            G[i:i + LV_WIN, j:j + LV_WIN] += (blk - blk.mean()) / ((N - LV_DDOF) * sd)
    return G / len(wins)


def image_prior_loss(S_masked, D, w_tv, w_lv):
    """w_tv TV(D S) + w_lv LV(D S) for masked coefficients S (n x a)."""
    X = D @ S_masked
    out = 0.0
    if w_tv:
        out += w_tv * tv_2d(X)
    if w_lv:
        out += w_lv * lv(X)
    return out


def image_prior_grad(S_masked, D, w_tv, w_lv):
    """Gradient of image_prior_loss with respect to S: D^T (dPrior/dX)."""
    X = D @ S_masked
    GX = np.zeros_like(X)
    if w_tv:
        GX += w_tv * tv_2d_grad(X)
    if w_lv:
        GX += w_lv * lv_grad(X)
    return D.T @ GX


def clomp_image_fp64(A, Y, k, params, w_tv=0.0, w_lv=0.0):
    """CLOMP on the a columns of Y (m x a) sharing A (m x n), with the image
    priors of Eq. (6)-(7) on X = D (Mask * S).  Returns a list of SolveResult,
    one per column, whose x is the learned coefficients (no refinement) and
    whose resid_norm is ||y_c - A x_c||; extra = {'steps', 'sigma'}."""
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    m, n = A.shape
    a = Y.shape[1]
    k_eff = min(k, m, n)
    T = params.inner_steps
    D = dct_synthesis(n) if (w_tv or w_lv) else None
    S = np.zeros((n, a))
    M = np.zeros((n, a))
    V = np.zeros((n, a))
    mask = np.zeros((n, a), dtype=bool)
    supports = [[] for _ in range(a)]
    gaps = [[] for _ in range(a)]
    status = [ST_K_CAPPED if k > k_eff else 0 for _ in range(a)]
    live = [float(np.linalg.norm(Y[:, c])) > 0.0 for c in range(a)]
    for c in range(a):
        if not live[c]:
            status[c] |= ST_ZERO_Y
    lr = np.zeros(a)
    eps = np.zeros(a)
    sigma = np.zeros(a)
    step = 0
    for t in range(k_eff):
        # residual injection and selection, column by column
        for c in range(a):
            if not live[c]:
                continue
            r = Y[:, c] - A @ np.where(mask[:, c], S[:, c], 0.0)
            cc = A.T @ r
            j, gap, nonfinite = argmax_unselected(cc, supports[c])
            if t == 0:
                sigma[c] = float(np.max(np.abs(cc)))
                eps[c] = params.eps_rel * sigma[c]
            lr[c] = params.lr_rel * float(abs(cc[j]))
            if nonfinite:
                status[c] |= ST_NAN
            gaps[c].append(gap)
            mask[j, c] = True
            supports[c].append(j)
        # T Adam steps on every column together
        for _ in range(T):
            step += 1
            Sm = np.where(mask, S, 0.0)
            G = np.where(mask, A.T @ (A @ Sm - Y), 0.0)
            if D is not None:
                G += np.where(mask, image_prior_grad(Sm, D, w_tv, w_lv), 0.0)
            for c in range(a):
                if not live[c]:
                    continue
                S[:, c], M[:, c], V[:, c] = adam_step_fp64(
                    S[:, c], G[:, c], M[:, c], V[:, c], step, lr[c], params.beta1,
                    params.beta2, eps[c])
    out = []
    for c in range(a):
        x = np.where(mask[:, c], S[:, c], 0.0)
        rn = float(np.linalg.norm(Y[:, c] - A @ x))
        out.append(SolveResult(supports[c], x, rn, gaps[c], [], status[c],
                               {"steps": step, "sigma": float(sigma[c])}))
    return out
