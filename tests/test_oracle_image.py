"""Pins of the image-prior oracle (Methods, Eq. (6), Eq. (7)) and of CLOMP on
the columns of an image, against closed forms, finite differences, an
independent torch rendering and reductions to the 1-D oracle."""

import math

import numpy as np
import pytest

from oracle import ClompParams, clomp_fp64, dct_synthesis, tv_1d
from oracle.image_prior import (clomp_image_fp64, image_prior_grad, image_prior_loss, lv,
                                lv_grad, tv_2d, tv_2d_grad)

f32 = lambda v: float(np.float32(v))
PARAMS = ClompParams(inner_steps=8, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                     eps_rel=f32(1e-8))


def _rng(i):
    return np.random.default_rng([2501, 11592, 66, i])


def test_tv2d_terms_match_eq5_per_column_and_parseval():
    """Eq. (6) = Eq. (5) on every column (the vertical term) + the horizontal
    term, which for X = D S with orthonormal D is (1/W) sum ||s_j - s_j+1||^2."""
    g = _rng(1)
    n, a = 24, 7
    D = dct_synthesis(n)
    S = g.standard_normal((n, a))
    X = D @ S
    vertical = sum(tv_1d(X[:, j]) for j in range(a))
    horizontal = sum(float(np.sum((S[:, j] - S[:, j + 1]) ** 2)) for j in range(a - 1)) / a
    assert abs(tv_2d(X) - (vertical + horizontal)) <= 1e-12 * tv_2d(X)


def test_tv2d_hand_example():
    """2 x 2 image [[1, 2], [4, 8]]: vertical (1-4)^2 + (2-8)^2 = 45 over H = 2,
    horizontal (1-2)^2 + (4-8)^2 = 17 over W = 2."""
    assert tv_2d(np.array([[1.0, 2.0], [4.0, 8.0]])) == 45 / 2 + 17 / 2


def test_tv2d_gradient_central_differences():
    """Eq. (6) is quadratic: central differences are exact up to rounding."""
    g = _rng(2)
    X = g.standard_normal((9, 6))
    G = tv_2d_grad(X)
    h = 1e-3
    for (i, j) in [(0, 0), (4, 2), (8, 5), (3, 0), (0, 5)]:
        E = np.zeros_like(X)
        E[i, j] = h
        fd = (tv_2d(X + E) - tv_2d(X - E)) / (2 * h)
        assert abs(fd - G[i, j]) <= 1e-9


def test_lv_closed_forms():
    """A constant image has LV = 0 and a zero gradient; a plane X = alpha i +
    beta j has the same window std everywhere, sqrt(6 (alpha^2 + beta^2) / 8),
    and that is LV."""
    C = np.full((7, 9), 3.25)
    assert lv(C) == 0.0 and not lv_grad(C).any()
    al, be = 0.7, -1.9
    i, j = np.meshgrid(np.arange(7.0), np.arange(9.0), indexing="ij")
    P = al * i + be * j
    assert abs(lv(P) - math.sqrt(6.0 * (al * al + be * be) / 8.0)) <= 1e-12
    # a 2 x 2 image holds no 3 x 3 window
    assert lv(np.ones((2, 5))) == 0.0


def test_lv_gradient_central_differences():
    g = _rng(3)
    X = g.standard_normal((8, 7))
    G = lv_grad(X)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 3), (7, 6), (4, 0), (2, 5)]:
        E = np.zeros_like(X)
        E[i, j] = h
        fd = (lv(X + E) - lv(X - E)) / (2 * h)
        assert abs(fd - G[i, j]) <= 1e-8


def test_lv_and_tv2d_match_torch_rendering():
    """An independent rendering: windows by torch's unfold, torch.std
    (unbiased) and autograd; Eq. (6) by tensor differences."""
    torch = pytest.importorskip("torch")
    g = _rng(4)
    X = g.standard_normal((10, 8))
    Xt = torch.tensor(X, requires_grad=True)
    win = torch.nn.functional.unfold(Xt[None, None], kernel_size=3, stride=1)[0]   # 9 x B
    lvt = win.std(dim=0, unbiased=True).mean()
    lvt.backward()
    assert abs(lvt.item() - lv(X)) <= 1e-12
    np.testing.assert_allclose(Xt.grad.numpy(), lv_grad(X), rtol=0, atol=1e-12)
    Xt2 = torch.tensor(X, requires_grad=True)
    tvt = ((Xt2[:-1] - Xt2[1:]) ** 2).sum() / X.shape[0] + \
        ((Xt2[:, :-1] - Xt2[:, 1:]) ** 2).sum() / X.shape[1]
    tvt.backward()
    assert abs(tvt.item() - tv_2d(X)) <= 1e-12
    np.testing.assert_allclose(Xt2.grad.numpy(), tv_2d_grad(X), rtol=0, atol=1e-12)


def test_prior_gradient_in_coefficients_chain_rule():
    """image_prior_grad = D^T (dPrior / dX): against central differences of
    image_prior_loss in the coefficients."""
    g = _rng(5)
    n, a = 12, 5
    D = dct_synthesis(n)
    S = g.standard_normal((n, a))
    G = image_prior_grad(S, D, 0.3, 0.7)
    h = 1e-6
    for (i, j) in [(0, 0), (5, 2), (11, 4), (3, 1)]:
        E = np.zeros_like(S)
        E[i, j] = h
        fd = (image_prior_loss(S + E, D, 0.3, 0.7) - image_prior_loss(S - E, D, 0.3, 0.7)) / (2 * h)
        assert abs(fd - G[i, j]) <= 1e-8


def _image_case(i, n=32, m=16, a=6, k=4):
    g = _rng(100 + i)
    A = g.standard_normal((m, n)) / math.sqrt(m)
    S = np.zeros((n, a))
    for c in range(a):
        S[g.choice(n, k, replace=False), c] = g.standard_normal(k)
    return A, A @ S, k


def test_image_clomp_without_priors_is_columnwise_clomp():
    """With w_tv = w_lv = 0 the columns decouple: each equals the 1-D oracle's
    support and its Adam iterate before the refinement."""
    A, Y, k = _image_case(0)
    res = clomp_image_fp64(A, Y, k, PARAMS)
    for c in range(Y.shape[1]):
        ref = clomp_fp64(A, Y[:, c], k, PARAMS)
        assert res[c].support == ref.support
        np.testing.assert_allclose(res[c].x[ref.support], ref.extra["s_adam"], rtol=1e-12,
                                   atol=1e-14)


def test_image_clomp_single_column_is_1d_tv_clomp():
    """One column (W = 1): Eq. (6) has no horizontal term and its vertical term
    is Eq. (5), so the image mode takes the 1-D TV oracle's Adam iterate."""
    A, Y, k = _image_case(1, a=1)
    w = 0.05
    res = clomp_image_fp64(A, Y, k, PARAMS, w_tv=w)
    from dataclasses import replace
    ref = clomp_fp64(A, Y[:, 0], k, replace(PARAMS, prior_tv=w))
    assert res[0].support == ref.support
    np.testing.assert_allclose(res[0].x[ref.support], ref.extra["s_adam"], rtol=1e-11,
                               atol=1e-13)


def test_image_clomp_column_reversal():
    """The priors are symmetric under a left-right flip of the image: reversing
    the columns of Y reverses the solution."""
    A, Y, k = _image_case(2)
    fwd = clomp_image_fp64(A, Y, k, PARAMS, w_tv=0.1, w_lv=0.05)
    rev = clomp_image_fp64(A, Y[:, ::-1], k, PARAMS, w_tv=0.1, w_lv=0.05)
    a = Y.shape[1]
    for c in range(a):
        assert fwd[c].support == rev[a - 1 - c].support
        np.testing.assert_allclose(fwd[c].x, rev[a - 1 - c].x, rtol=0, atol=1e-12)


def test_image_clomp_matches_torch_autograd_and_adam():
    """Independent rendering: the whole image loss by torch autograd on a
    masked parameter per column, torch.optim.Adam with one parameter group per
    column (its own lr and eps), argmax selection per column from its own
    residual."""
    torch = pytest.importorskip("torch")
    A, Y, k = _image_case(3)
    w_tv, w_lv = 0.2, 0.1
    res = clomp_image_fp64(A, Y, k, PARAMS, w_tv=w_tv, w_lv=w_lv)
    m, n = A.shape
    a = Y.shape[1]
    At = torch.tensor(A)
    Yt = torch.tensor(Y)
    Dt = torch.tensor(dct_synthesis(n))
    params = [torch.zeros(n, dtype=torch.float64, requires_grad=True) for _ in range(a)]
    masks = [torch.zeros(n, dtype=torch.float64) for _ in range(a)]
    supports = [[] for _ in range(a)]
    opt = None
    sig = [None] * a
    for t in range(k):
        lrs = []
        for c in range(a):
            with torch.no_grad():
                r = Yt[:, c] - At @ (masks[c] * params[c])
                cc = (At.T @ r).abs()
                cc[supports[c]] = -1.0
                j = int(torch.argmax(cc))
                if t == 0:
                    sig[c] = float((At.T @ Yt[:, c]).abs().max())
                lrs.append(PARAMS.lr_rel * float(cc[j]))
            supports[c].append(j)
            masks[c][j] = 1.0
        if opt is None:
            opt = torch.optim.Adam([{"params": [p], "lr": lrs[c], "eps": PARAMS.eps_rel * sig[c]}
                                    for c, p in enumerate(params)],
                                   betas=(PARAMS.beta1, PARAMS.beta2), foreach=False)
        else:
            for c, grp in enumerate(opt.param_groups):
                grp["lr"] = lrs[c]
        for _ in range(PARAMS.inner_steps):
            opt.zero_grad()
            Sm = torch.stack([masks[c] * params[c] for c in range(a)], dim=1)
            X = Dt @ Sm
            fit = 0.5 * ((At @ Sm - Yt) ** 2).sum()
            tv = ((X[:-1] - X[1:]) ** 2).sum() / n + ((X[:, :-1] - X[:, 1:]) ** 2).sum() / a
            win = torch.nn.functional.unfold(X[None, None], kernel_size=3, stride=1)[0]
            lvv = win.std(dim=0, unbiased=True).mean()
            (fit + w_tv * tv + w_lv * lvv).backward()
            opt.step()
    for c in range(a):
        assert res[c].support == supports[c]
        xt = (masks[c] * params[c]).detach().numpy()
        np.testing.assert_allclose(res[c].x, xt, rtol=0, atol=1e-10 * np.abs(xt).max())
