"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself or with the GPU path: each check
uses a hand-derived value, a closed form, a textbook invariant, an independent
library routine (LAPACK SVD least squares, scikit-learn's OMP, torch autograd
and torch.optim.Adam) or brute force.
"""

import math
import os

import numpy as np
import pytest

from oracle import (omp_fp64, clomp_fp64, ClompParams, clomp_paper_fp64, PaperParams,
                    omp_cgs2_fp64, clomp_gram_fp64, separation_report, separated_prefix,
                    common_prefix, perturbed_atoms, perturbed_vector,
                    iht_fp64, lstsq_support,
                    resid_norm_fp64, grad_fp64, adam_step_fp64,
                    bruteforce_support, well_separated,
                    dct_synthesis, forward_difference, tv_1d, tv_grad_coeffs, lstsq_support_tv)
from oracle.omp import ST_ZERO_Y, ST_K_CAPPED, ST_NAN, ST_EARLY_STOP
from paper_2501_11592_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse_golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([f.strip() for f in line.split("|")])
    return rows


def _vec(s):
    return np.array([float(v) for v in s.split()]) if s.strip() else np.zeros(0)


def _mat_rows(s):
    return np.array([[float(v) for v in r.split()] for r in s.split(";")])


def gaussian_instance(seed, m, n, k):
    """Noiseless k-sparse Gaussian instance in float64 (y computed in float64)."""
    g = np.random.default_rng([99, seed, m, n, k])
    A = g.standard_normal((m, n)) / math.sqrt(m)
    supp = np.sort(g.choice(n, size=k, replace=False))
    s = np.zeros(n)
    s[supp] = g.standard_normal(k)
    return A, A @ s, supp, s


# ------------------------------------------------------------------ golden
@pytest.mark.parametrize("row", _parse_golden("omp_worked_examples.txt"),
                         ids=lambda r: r[0])
def test_omp_worked_examples(row):
    _, cols, y, k, supp, x, rn = row
    A = _mat_rows(cols).T
    y = _vec(y)
    res = omp_fp64(A, y, int(k))
    assert res.support == [int(v) for v in supp.split()]
    np.testing.assert_allclose(res.x, _vec(x), rtol=0, atol=1e-14)
    assert abs(res.resid_norm - float(rn)) < 1e-14
    # CLOMP selects the same atoms here and refines to the same least squares
    cres = clomp_fp64(A, y, int(k), ClompParams(inner_steps=64))
    assert cres.support == res.support
    np.testing.assert_allclose(cres.x, _vec(x), rtol=0, atol=1e-14)


@pytest.mark.parametrize("row", _parse_golden("grad_worked_example.txt"),
                         ids=lambda r: r[0])
def test_grad_worked_example(row):
    _, Arows, x, mask, y, loss, grad = row
    l, g, _ = grad_fp64(_vec(x), _vec(mask), _mat_rows(Arows), _vec(y))
    assert l == float(loss)
    np.testing.assert_array_equal(g, _vec(grad))


# ------------------------------------------------------------------ O6 / a7
def test_lstsq_matches_svd_lstsq_and_normal_equations():
    A, y, _, _ = gaussian_instance(1, 40, 100, 6)
    y = y + np.random.default_rng(3).standard_normal(40) * 0.1
    S = [5, 17, 3, 88, 41, 60, 12]
    xq = lstsq_support(A, y, S)
    xs = np.linalg.lstsq(A[:, S], y, rcond=None)[0]
    np.testing.assert_allclose(xq, xs, rtol=1e-12, atol=1e-13)
    r = y - A[:, S] @ xq
    assert np.max(np.abs(A[:, S].T @ r)) < 1e-12 * np.linalg.norm(A[:, S]) * np.linalg.norm(y)
    assert abs(resid_norm_fp64(A, y, S, xq) - math.sqrt(float(r @ r))) < 1e-15 * (1 + np.linalg.norm(y))
    assert resid_norm_fp64(A, y, [], []) == pytest.approx(np.linalg.norm(y), rel=1e-15)


# ------------------------------------------------------------------ O3 brute force
def test_bruteforce_finds_planted_support():
    A, y, supp, _ = gaussian_instance(2, 8, 14, 3)
    best, r, table = bruteforce_support(A, y, 3)
    assert best == list(supp) and r < 1e-12
    assert len(table) == math.comb(14, 3)


@pytest.mark.parametrize("seed", range(12))
def test_omp_never_beats_bruteforce_and_matches_on_recoverable(seed):
    g = np.random.default_rng([5, seed])
    m, n, k = 7, int(g.integers(10, 17)), int(g.integers(1, 4))
    A, y, supp, _ = gaussian_instance(seed, m, n, k)
    noisy = y + 0.3 * g.standard_normal(m)
    for yy in (y, noisy):
        best, rbf, _ = bruteforce_support(A, yy, k)
        res = omp_fp64(A, yy, k)
        assert res.resid_norm >= rbf - 1e-12
        if yy is y and sorted(res.support) == list(supp):
            assert sorted(res.support) == best


# ------------------------------------------------------------------ O1 OMP
def test_omp_exact_recovery_rate_and_accuracy():
    recovered = 0
    for seed in range(30):
        A, y, supp, s = gaussian_instance(seed, 64, 256, 8)
        res = omp_fp64(A, y, 8)
        if sorted(res.support) == list(supp):
            recovered += 1
            assert np.max(np.abs(res.x - s)) < 1e-10
    assert recovered >= 28          # OMP recovers m/k = 8 Gaussian instances w.h.p.


def test_omp_residual_orthogonal_and_monotone():
    A, y, _, _ = gaussian_instance(7, 50, 200, 10)
    y = y + 0.05 * np.random.default_rng(1).standard_normal(50)
    res = omp_fp64(A, y, 20)
    hist = [np.linalg.norm(y)] + res.resid_hist
    assert all(b <= a * (1 + 1e-14) for a, b in zip(hist, hist[1:]))
    # invariant after the last step (every intermediate step re-solves from scratch)
    for t in range(1, len(res.support) + 1):
        S = res.support[:t]
        xS = lstsq_support(A, y, S)
        r = y - A[:, S] @ xS
        assert np.max(np.abs(A[:, S].T @ r)) <= 1e-10 * np.linalg.norm(A[:, S]) * np.linalg.norm(y)


def test_omp_full_support_zero_residual():
    A, y, _, _ = gaussian_instance(11, 12, 30, 4)
    y = y + np.random.default_rng(2).standard_normal(12)
    res = omp_fp64(A, y, 12)
    assert len(res.support) == 12 and res.resid_norm < 1e-12 * np.linalg.norm(y)


def test_omp_matches_sklearn_on_well_separated():
    from sklearn.linear_model import orthogonal_mp
    checked = 0
    for seed in range(20):
        A, y, _, _ = gaussian_instance(seed, 64, 256, 8)
        y = y + 0.01 * np.random.default_rng(seed).standard_normal(64)
        ok, res = well_separated(A, y, 8, method="omp", delta=1e-3)
        if not ok:
            continue
        checked += 1
        coef = orthogonal_mp(A, y, n_nonzero_coefs=8)
        assert sorted(np.flatnonzero(coef).tolist()) == sorted(res.support)
        np.testing.assert_allclose(res.x, coef, rtol=0, atol=1e-10)
    assert checked >= 10


def test_omp_flags():
    A, y, _, _ = gaussian_instance(3, 6, 20, 2)
    r = omp_fp64(A, np.zeros(6), 3)
    assert r.status & ST_ZERO_Y and r.support == [] and not r.x.any()
    r = omp_fp64(A, y, 9)
    assert r.status & ST_K_CAPPED and len(r.support) == 6
    yn = y.copy()
    yn[2] = np.nan
    assert omp_fp64(A, yn, 2).status & ST_NAN
    r = omp_fp64(A, y, 6, resid_tol=1e-9)
    assert r.status & ST_EARLY_STOP and len(r.support) < 6
    assert r.resid_norm <= 1e-9 * np.linalg.norm(y)


# ------------------------------------------------------------------ O4 / O5
def test_grad_central_differences_exact_for_quadratic():
    A, y, _, _ = gaussian_instance(4, 9, 15, 3)
    g = np.random.default_rng(8)
    x = g.standard_normal(15)
    mask = g.random(15) < 0.5
    _, grad, _ = grad_fp64(x, mask, A, y)
    h = 1e-3
    for j in range(15):
        e = np.zeros(15)
        e[j] = h
        lp = grad_fp64(x + e, mask, A, y)[0]
        lm = grad_fp64(x - e, mask, A, y)[0]
        assert abs((lp - lm) / (2 * h) - grad[j]) < 1e-9
    assert not grad[~mask].any()


def test_grad_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    A, y, _, _ = gaussian_instance(5, 11, 23, 3)
    g = np.random.default_rng(9)
    x = g.standard_normal(23)
    mask = (g.random(23) < 0.6).astype(np.float64)
    xt = torch.tensor(x, requires_grad=True)
    loss = 0.5 * ((torch.tensor(A) @ (torch.tensor(mask) * xt) - torch.tensor(y)) ** 2).sum()
    loss.backward()
    l, gr, _ = grad_fp64(x, mask, A, y)
    assert abs(l - loss.item()) <= 1e-14 * abs(l)
    np.testing.assert_allclose(gr, xt.grad.numpy(), rtol=1e-13, atol=1e-14)


def test_adam_matches_torch_optim_adam():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(10)
    grads = [g.standard_normal(7) * (1 + 10 * (i % 3)) for i in range(50)]
    grads[5][2] = 0.0
    p = torch.zeros(7, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.03, betas=(0.9, 0.999), eps=1e-6, foreach=False)
    th, m, v = np.zeros(7), np.zeros(7), np.zeros(7)
    for i, gr in enumerate(grads):
        p.grad = torch.tensor(gr)
        opt.step()
        th, m, v = adam_step_fp64(th, gr, m, v, i + 1, 0.03, 0.9, 0.999, 1e-6)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_adam_zero_gradient_coordinates_do_not_move():
    th, m, v = adam_step_fp64(np.array([1.5, -2.0]), np.array([0.0, 3.0]),
                              np.zeros(2), np.zeros(2), 1, 0.1, 0.9, 0.999, 1e-8)
    assert th[0] == 1.5 and m[0] == 0.0 and v[0] == 0.0


# ------------------------------------------------------------------ O2 CLOMP
def test_clomp_exact_inner_reduces_to_omp():
    for seed in range(6):
        A, y, _, _ = gaussian_instance(seed, 30, 90, 6)
        y = y + 0.02 * np.random.default_rng(seed).standard_normal(30)
        a = omp_fp64(A, y, 8)
        b = clomp_fp64(A, y, 8, inner="exact")
        assert a.support == b.support
        np.testing.assert_allclose(a.x, b.x, rtol=0, atol=1e-14)
        assert abs(a.resid_norm - b.resid_norm) < 1e-14


def test_clomp_orthonormal_dictionary_closed_form():
    """With orthonormal columns the correlation of an unselected column is
    a_j^T y whatever s is, so CLOMP selects the k largest |a_j^T y| in
    decreasing order and refines to x_S = A_S^T y, for any Adam trajectory."""
    g = np.random.default_rng(12)
    Q, _ = np.linalg.qr(g.standard_normal((20, 20)))
    y = g.standard_normal(20)
    c = Q.T @ y
    order = list(np.argsort(-np.abs(c), kind="stable")[:7])
    for T in (1, 3, 32):
        res = clomp_fp64(Q, y, 7, ClompParams(inner_steps=T))
        assert res.support == [int(j) for j in order]
        np.testing.assert_allclose(res.x[order], c[order], rtol=0, atol=1e-13)
        assert not np.delete(res.x, order).any()


def test_clomp_first_adam_step_closed_form():
    """From s = m = v = 0 the first Adam step on the single selected column j
    moves s_j by lr * c_j / (|c_j| + eps), with g = -c_j."""
    A, y, _, _ = gaussian_instance(13, 10, 40, 3)
    p = ClompParams(inner_steps=1, lr_rel=0.05, eps_rel=1e-3)
    res = clomp_fp64(A, y, 1, p)
    c = A.T @ y
    j = int(np.argmax(np.abs(c)))
    sigma = abs(c[j])
    lr, eps = 0.05 * sigma, 1e-3 * sigma
    assert res.support == [j]
    assert abs(res.extra["s_adam"][0] - lr * c[j] / (abs(c[j]) + eps)) < 1e-15 * sigma


def test_clomp_matches_autograd_and_torch_adam_rendering():
    """Independent rendering of the paper's CLOMP with framework pieces: s is a
    torch parameter of n entries, the forward is A (mask * s), the loss is
    1/2 ||y' - y||^2, backward by autograd, update by torch.optim.Adam with a
    per-iteration learning rate 0.05 |c_j|."""
    torch = pytest.importorskip("torch")
    for seed in range(3):
        A, y, _, _ = gaussian_instance(seed, 16, 48, 4)
        y = y + 0.01 * np.random.default_rng(seed).standard_normal(16)
        P = ClompParams(inner_steps=12, lr_rel=0.05)
        ref = clomp_fp64(A, y, 5, P)
        At, yt = torch.tensor(A), torch.tensor(y)
        s = torch.zeros(48, dtype=torch.float64, requires_grad=True)
        mask = torch.zeros(48, dtype=torch.float64)
        opt = None
        S = []
        for t in range(5):
            with torch.no_grad():
                c = At.T @ (yt - At @ (mask * s))
                score = c.abs().clone()
                score[mask.bool()] = -float("inf")
                j = int(torch.argmax(score))
                if t == 0:
                    sig = float(c.abs().max())
                    opt = torch.optim.Adam([s], lr=0.05 * sig, betas=(0.9, 0.999),
                                           eps=1e-8 * sig, foreach=False)
                # learning-rate schedule: lr follows the selected correlation
                opt.param_groups[0]["lr"] = 0.05 * abs(float(c[j]))
                mask[j] = 1.0
                S.append(j)
            for _ in range(12):
                opt.zero_grad()
                loss = 0.5 * ((At @ (mask * s) - yt) ** 2).sum()
                loss.backward()
                opt.step()
        assert S == ref.support
        np.testing.assert_allclose(s.detach().numpy()[S], ref.extra["s_adam"],
                                   rtol=1e-11, atol=1e-13)


def test_clomp_power_of_two_scaling_equivariance():
    A, y, _, _ = gaussian_instance(14, 32, 128, 6)
    y = y + 0.01 * np.random.default_rng(0).standard_normal(32)
    a = clomp_fp64(A, y, 8)
    for p in (-7, 3, 20):
        b = clomp_fp64(A, y * 2.0 ** p, 8)
        assert b.support == a.support
        np.testing.assert_array_equal(b.extra["s_adam"], a.extra["s_adam"] * 2.0 ** p)
        np.testing.assert_allclose(b.x, a.x * 2.0 ** p, rtol=1e-14, atol=0)


def test_clomp_column_permutation_equivariance():
    A, y, _, _ = gaussian_instance(15, 24, 80, 5)
    perm = np.random.default_rng(4).permutation(80)
    a = clomp_fp64(A, y, 6)
    b = clomp_fp64(A[:, perm], y, 6)
    assert [int(perm[j]) for j in b.support] == a.support
    np.testing.assert_allclose(b.x, a.x[perm], rtol=0, atol=1e-12)


def test_clomp_exact_recovery_noiseless():
    recovered = 0
    for seed in range(20):
        A, y, supp, s = gaussian_instance(seed, 64, 256, 8)
        res = clomp_fp64(A, y, 8)
        if sorted(res.support) == list(supp):
            recovered += 1
            assert np.max(np.abs(res.x - s)) < 1e-10
            assert res.resid_norm < 1e-12
    assert recovered >= 17


def test_clomp_bf16_style_refinement_uses_master():
    """Selection on a perturbed copy, refinement on the master: the final x is
    the master least squares on the selected support."""
    A, y, _, _ = gaussian_instance(16, 40, 120, 5)
    Ab = A * (1 + 2.0 ** -8 * np.random.default_rng(1).choice([-1, 1], A.shape))
    res = clomp_fp64(Ab, y, 5, A_refine=A)
    np.testing.assert_allclose(res.x[res.support], lstsq_support(A, y, res.support),
                               rtol=0, atol=1e-14)
    assert abs(res.resid_norm - resid_norm_fp64(A, y, res.support, res.x[res.support])) < 1e-15


def test_clomp_flags():
    A, y, _, _ = gaussian_instance(17, 6, 20, 2)
    r = clomp_fp64(A, np.zeros(6), 3)
    assert r.status & ST_ZERO_Y and r.support == []
    r = clomp_fp64(A, y, 10)
    assert r.status & ST_K_CAPPED and len(r.support) == 6


# ---------------------------------------------------------------- F1 paper mode
def test_paper_mode_matches_autograd_and_torch_adam_rendering():
    """Independent rendering of paper-mode CLOMP with framework pieces: the
    normalised scores |c| / max|c| cut at T_h, the mask OR-ed, then one
    autograd backward of 1/2 ||A(mask*s) - y||^2 and one torch.optim.Adam step
    per iteration with lr = lr_rel * max|c|."""
    torch = pytest.importorskip("torch")
    for seed in range(3):
        A, y, _, _ = gaussian_instance(40 + seed, 24, 64, 4)
        y = y + 0.01 * np.random.default_rng(seed).standard_normal(24)
        P = PaperParams(threshold=0.6, max_iters=25, lr_rel=0.1)
        ref = clomp_paper_fp64(A, y, 24, P)
        At, yt = torch.tensor(A), torch.tensor(y)
        s = torch.zeros(64, dtype=torch.float64, requires_grad=True)
        mask = torch.zeros(64, dtype=torch.bool)
        opt = None
        for it in range(25):
            with torch.no_grad():
                c = At.T @ (yt - At @ torch.where(mask, s, torch.zeros_like(s)))
                cmax = float(c.abs().max())
                if it == 0:
                    opt = torch.optim.Adam([s], lr=0.1 * cmax, betas=(0.9, 0.999),
                                           eps=1e-8 * cmax, foreach=False)
                opt.param_groups[0]["lr"] = 0.1 * cmax
                new = (~mask) & (c.abs() / cmax >= 0.6)
                if int(mask.sum()) + int(new.sum()) <= 24:
                    mask |= new
            opt.zero_grad()
            loss = 0.5 * ((At @ torch.where(mask, s, torch.zeros_like(s)) - yt) ** 2).sum()
            loss.backward()
            opt.step()
        S = torch.nonzero(mask).flatten().tolist()
        assert S == ref.support
        np.testing.assert_allclose(s.detach().numpy()[S], ref.extra["s_adam"],
                                   rtol=1e-11, atol=1e-13)


def test_paper_mode_orthonormal_first_batch_closed_form():
    """A orthonormal (m = n) and y = A s: c = A^T y = s at the first
    iteration, so the first batch is { j : |s_j| >= T_h max|s| }."""
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    strue = rng.standard_normal(40) * (rng.random(40) < 0.3)
    res = clomp_paper_fp64(Q, Q @ strue, 40, PaperParams(threshold=0.5, max_iters=1))
    expect = np.flatnonzero(np.abs(strue) >= 0.5 * np.abs(strue).max()).tolist()
    assert res.extra["batches"] == [expect] and res.support == expect


def test_paper_mode_power_of_two_scaling_and_invariants():
    A, y, _, _ = gaussian_instance(44, 32, 128, 6)
    y = y + 0.01 * np.random.default_rng(1).standard_normal(32)
    P = PaperParams(max_iters=60)
    a = clomp_paper_fp64(A, y, 10, P)
    for p in (-5, 9):
        b = clomp_paper_fp64(A, y * 2.0 ** p, 10, P)
        assert b.support == a.support
        np.testing.assert_array_equal(b.extra["s_adam"], a.extra["s_adam"] * 2.0 ** p)
    # the support is the union of the accepted batches, within k_eff, and a
    # refused batch sets the K-capped bit
    union = sorted(j for bt in a.extra["batches"] for j in bt)
    assert union == a.support and len(a.support) <= 10
    full = clomp_paper_fp64(A, y, 32, P)
    assert len(full.support) >= len(a.support)
    if len(a.support) < len(full.support):
        assert a.status & ST_K_CAPPED


# ---------------------------------------------------------------- F4 IHT
def test_iht_top_k_ties_and_nan():
    from oracle.iht import top_k
    z = np.array([1.0, -3.0, 3.0, 0.5, np.nan, -1.0, 3.0])
    sel, _ = top_k(z, 3)        # NaN first, then |3| at indices 1, 2 (lowest of three)
    assert sel.tolist() == [1, 2, 4]
    sel, gap = top_k(np.array([4.0, -2.0, 1.0]), 2)
    assert sel.tolist() == [0, 1] and gap == pytest.approx(0.5)


def test_iht_orthonormal_closed_form():
    """A orthonormal: the normalised step is exactly 1 and one iteration
    lands on H_K(A^T y) = H_K(s), a fixed point of every later iteration."""
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    strue = rng.standard_normal(50)
    y = Q @ strue
    K = 7
    expect = np.sort(np.argsort(-np.abs(strue), kind="stable")[:K])
    for R in (1, 6):
        res = iht_fp64(Q, y, K, max_iters=R)
        assert res.support == expect.tolist()
        np.testing.assert_allclose(res.extra["s_iht"], strue[expect], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(res.extra["steps"], 1.0, rtol=1e-12)


def test_iht_exact_recovery_noiseless():
    """Noiseless Gaussian k-sparse instances (n=256, m=64, k=8): the k-sparse
    solution is unique and normalised IHT reaches it."""
    ok = 0
    for seed in range(20):
        sig = W.single_small(900 + seed)
        res = iht_fp64(sig.A, sig.y, 8)
        if res.support == sig.support.tolist():
            ok += 1
            np.testing.assert_allclose(res.x, sig.s, rtol=0, atol=1e-7)
    assert ok >= 19


def test_iht_matches_autograd_and_torch_topk_rendering():
    """Independent rendering: the gradient of 1/2||As - y||^2 by autograd and
    the hard threshold by a stable descending torch sort."""
    torch = pytest.importorskip("torch")
    for seed in range(3):
        A, y, _, _ = gaussian_instance(60 + seed, 30, 90, 5)
        y = y + 0.01 * np.random.default_rng(seed).standard_normal(30)
        ref = iht_fp64(A, y, 6, max_iters=15)
        At, yt = torch.tensor(A), torch.tensor(y)
        s = torch.zeros(90, dtype=torch.float64)
        G = None
        for it in range(15):
            sv = s.clone().requires_grad_(True)
            loss = 0.5 * ((At @ sv - yt) ** 2).sum()
            loss.backward()
            g = -sv.grad
            if G is None:
                G = torch.sort(torch.sort(-g.abs(), stable=True).indices[:6]).values
            gG = g[G]
            t = float((gG ** 2).sum() / ((At[:, G] @ gG) ** 2).sum())
            z = s + t * g
            G = torch.sort(torch.sort(-z.abs(), stable=True).indices[:6]).values
            s = torch.zeros(90, dtype=torch.float64)
            s[G] = z[G]
        assert G.tolist() == ref.support
        np.testing.assert_allclose(s[G].numpy(), ref.extra["s_iht"], rtol=1e-10, atol=1e-13)


def test_iht_power_of_two_scaling_and_permutation():
    A, y, _, _ = gaussian_instance(64, 32, 128, 6)
    y = y + 0.01 * np.random.default_rng(2).standard_normal(32)
    a = iht_fp64(A, y, 6, max_iters=40)
    b = iht_fp64(A, y * 2.0 ** 7, 6, max_iters=40)
    assert b.support == a.support
    np.testing.assert_array_equal(b.extra["s_iht"], a.extra["s_iht"] * 2.0 ** 7)
    perm = np.random.default_rng(3).permutation(128)
    c = iht_fp64(A[:, perm], y, 6, max_iters=40)
    assert sorted(int(perm[j]) for j in c.support) == a.support
    np.testing.assert_allclose(c.x, a.x[perm], rtol=0, atol=1e-10)


def test_workload_generators_are_deterministic():
    a = W.single_small(3)
    b = W.single_small(3)
    np.testing.assert_array_equal(a.At, b.At)
    np.testing.assert_array_equal(a.y, b.y)
    assert a.At.shape == (256, 64) and a.At.dtype == np.float32
    sb = W.image_batch(0.1)
    assert sb.m == 26 and sb.At.shape == (256, 32) and sb.Y.shape == (256, 26)
    assert not sb.At[:, 26:].any()
    specs = W.uneven_specs(64)
    for sp in specs:
        assert 512 <= sp.n <= 8192 and 0.09 * sp.n <= sp.m <= 0.51 * sp.n
        assert math.ceil(sp.n / 64) <= sp.k <= sp.n // 16


# ---------------------------------------------------------------- F2 TV prior
# Eq. (5): TV(x) = (1/n) sum (x_j - x_{j+1})^2 on x = D s, D the DCT basis.

def test_dct_synthesis_is_scipy_orthonormal_idct():
    """Library special case: column k of D is the inverse orthonormal DCT-II of
    the k-th unit vector; D is orthogonal."""
    sfft = pytest.importorskip("scipy.fft")
    for n in (1, 2, 7, 64, 255):
        D = dct_synthesis(n)
        ref = sfft.idct(np.eye(n), type=2, norm="ortho", axis=0)
        np.testing.assert_allclose(D, ref, rtol=0, atol=1e-13)
        np.testing.assert_allclose(D.T @ D, np.eye(n), rtol=0, atol=1e-12)


def test_tv_of_dct_coefficients_closed_form():
    """The DCT-II basis diagonalises the path-graph difference operator:
    TV(D s) = (1/n) sum_k 4 sin^2(pi k / (2n)) s_k^2, and the gradient is
    (2/n) * 4 sin^2(pi k / (2n)) s_k (an identity of the mathematics, not of
    the oracle's explicit differences)."""
    rng = np.random.default_rng(3)
    for n in (2, 9, 128, 333):
        s = rng.standard_normal(n)
        lam = 4.0 * np.sin(np.pi * np.arange(n) / (2.0 * n)) ** 2
        D = dct_synthesis(n)
        assert abs(tv_1d(D @ s) - np.sum(lam * s * s) / n) <= 1e-12 * (1 + np.sum(s * s))
        np.testing.assert_allclose(tv_grad_coeffs(s, D), (2.0 / n) * lam * s, rtol=0,
                                   atol=1e-12 * np.abs(s).max())
    # hand example: n = 3, x = (1, 0, 2): TV = (1 + 4) / 3
    assert abs(tv_1d(np.array([1.0, 0.0, 2.0])) - 5.0 / 3.0) < 1e-15
    np.testing.assert_array_equal(forward_difference(3),
                                  np.array([[1.0, -1.0, 0.0], [0.0, 1.0, -1.0]]))


def test_tv_prior_gradient_central_differences():
    """The prior loss is quadratic in s: central differences are exact up to
    rounding for the full loss 1/2||y - A(mask*s)||^2 + w TV(D(mask*s))."""
    A, y, _, _ = gaussian_instance(31, 12, 40, 3)
    rng = np.random.default_rng(5)
    mask = np.zeros(40, dtype=bool)
    mask[[2, 7, 19, 33]] = True
    s = rng.standard_normal(40)
    w = 0.37
    D = dct_synthesis(40)

    def loss(v):
        vm = np.where(mask, v, 0.0)
        return 0.5 * np.sum((A @ vm - y) ** 2) + w * tv_1d(D @ vm)

    sm = np.where(mask, s, 0.0)
    g = np.where(mask, A.T @ (A @ sm - y) + w * tv_grad_coeffs(sm, D), 0.0)
    h = 1e-3
    for j in range(40):
        e = np.zeros(40)
        e[j] = h
        fd = (loss(s + e) - loss(s - e)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-9 * (1 + abs(g[j])), (j, fd, g[j])


def test_clomp_prior_zero_weight_is_clomp():
    A, y, _, _ = gaussian_instance(32, 24, 80, 5)
    a = clomp_fp64(A, y, 6)
    b = clomp_fp64(A, y, 6, ClompParams(prior_tv=0.0))
    assert a.support == b.support
    np.testing.assert_array_equal(a.extra["s_adam"], b.extra["s_adam"])
    np.testing.assert_array_equal(a.x, b.x)


def test_clomp_prior_refinement_solves_regularised_normal_equations():
    """The refinement with the prior is the minimiser of the prior loss on the
    support: (A_S^T A_S + w (2/n) (Delta D_S)^T (Delta D_S)) x = A_S^T y."""
    A, y, _, _ = gaussian_instance(33, 20, 64, 4)
    y = y + 0.05 * np.random.default_rng(1).standard_normal(20)
    w = 2.5
    res = clomp_fp64(A, y, 6, ClompParams(prior_tv=w))
    S = res.support
    D = dct_synthesis(64)
    B = forward_difference(64) @ D[:, S]
    lhs = A[:, S].T @ A[:, S] + w * (2.0 / 64) * B.T @ B
    np.testing.assert_allclose(lhs @ res.x[S], A[:, S].T @ y, rtol=0, atol=1e-11)
    # the prior pulls the fit away from the plain least squares
    assert np.linalg.norm(res.x[S] - lstsq_support(A, y, S)) > 1e-6
    np.testing.assert_allclose(lstsq_support_tv(A, y, S, w, D), res.x[S], rtol=0, atol=1e-13)


def test_clomp_prior_matches_autograd_and_torch_adam_rendering():
    """Independent rendering with framework pieces: the loss adds w * TV of the
    signal D (mask * s) written with torch differences; autograd and
    torch.optim.Adam as in the plain rendering."""
    torch = pytest.importorskip("torch")
    sfft = pytest.importorskip("scipy.fft")
    for seed in range(2):
        A, y, _, _ = gaussian_instance(40 + seed, 16, 48, 4)
        y = y + 0.01 * np.random.default_rng(seed).standard_normal(16)
        w = 0.8
        P = ClompParams(inner_steps=12, lr_rel=0.05, prior_tv=w)
        ref = clomp_fp64(A, y, 5, P)
        At, yt = torch.tensor(A), torch.tensor(y)
        Dt = torch.tensor(sfft.idct(np.eye(48), type=2, norm="ortho", axis=0))
        s = torch.zeros(48, dtype=torch.float64, requires_grad=True)
        mask = torch.zeros(48, dtype=torch.float64)
        opt = None
        S = []
        for t in range(5):
            with torch.no_grad():
                c = At.T @ (yt - At @ (mask * s))
                score = c.abs().clone()
                score[mask.bool()] = -float("inf")
                j = int(torch.argmax(score))
                if t == 0:
                    sig = float(c.abs().max())
                    opt = torch.optim.Adam([s], lr=0.05 * sig, betas=(0.9, 0.999),
                                           eps=1e-8 * sig, foreach=False)
                opt.param_groups[0]["lr"] = 0.05 * abs(float(c[j]))
                mask[j] = 1.0
                S.append(j)
            for _ in range(12):
                opt.zero_grad()
                xs = Dt @ (mask * s)
                loss = 0.5 * ((At @ (mask * s) - yt) ** 2).sum() + \
                    w * ((xs[:-1] - xs[1:]) ** 2).sum() / 48
                loss.backward()
                opt.step()
        assert S == ref.support
        np.testing.assert_allclose(s.detach().numpy()[S], ref.extra["s_adam"],
                                   rtol=1e-10, atol=1e-12)


# ------------------------------------------------- large-instance renderings
# omp_cgs2_fp64 / clomp_gram_fp64 compute O1 / O2 through exact identities
# (updated QR; G_S s_S - b_S).  Pinned against the plain renderings, which are
# pinned above, and the Gram form also against the autograd rendering.

def _instances():
    out = []
    for seed in range(4):
        A, y, _, _ = gaussian_instance(40 + seed, 64, 256, 8)
        out.append((A, y + 0.01 * np.random.default_rng(seed).standard_normal(64), 10))
    A, y, _, _ = gaussian_instance(50, 160, 600, 40)
    out.append((A, y + 1e-3 * np.random.default_rng(9).standard_normal(160), 48))
    g = np.random.default_rng(51)
    A = g.standard_normal((120, 480)) / math.sqrt(120)
    supp, s = W.power_law_coeffs(g, 480, 60)
    out.append((A, A @ s, 60))
    return out


def test_incremental_omp_matches_plain_omp():
    for A, y, k in _instances():
        At = np.ascontiguousarray(A.T)            # atom-major storage, passed as a view
        a = omp_fp64(A, y, k)
        b = omp_cgs2_fp64(At.T, y, k)
        assert b.support == a.support
        np.testing.assert_allclose(b.x, a.x, rtol=0, atol=1e-10 * np.abs(a.x).max())
        assert abs(b.resid_norm - a.resid_norm) <= 1e-10 * np.linalg.norm(y)
        np.testing.assert_allclose(b.gaps, a.gaps, rtol=1e-6, atol=1e-12)


def test_incremental_omp_refines_on_master():
    A, y, _ = _instances()[4]
    Ab = A * (1 + 2.0 ** -8 * np.random.default_rng(3).choice([-1, 1], A.shape))
    r = omp_cgs2_fp64(Ab, y, 30, A_refine=A)
    assert r.support == omp_fp64(Ab, y, 30).support
    np.testing.assert_allclose(r.x[r.support], lstsq_support(A, y, r.support), rtol=0,
                               atol=1e-13)


def test_gram_clomp_matches_plain_clomp():
    for A, y, k in _instances():
        At = np.ascontiguousarray(A.T)
        a = clomp_fp64(A, y, k)
        b = clomp_gram_fp64(At.T, y, k, ClompParams())
        assert b.support == a.support
        sa = a.extra["s_adam"]
        np.testing.assert_allclose(b.extra["s_adam"], sa, rtol=0, atol=1e-10 * np.abs(sa).max())
        np.testing.assert_allclose(b.x, a.x, rtol=0, atol=1e-10 * np.abs(a.x).max())
        assert b.extra["steps"] == a.extra["steps"]
        assert abs(b.extra["sigma"] - a.extra["sigma"]) <= 1e-14 * a.extra["sigma"]
        assert abs(b.resid_norm - a.resid_norm) <= 1e-10 * np.linalg.norm(y)


def test_gram_clomp_bf16_style_with_master_matches_plain():
    A, y, _ = _instances()[4]
    Ab = A * (1 + 2.0 ** -8 * np.random.default_rng(5).choice([-1, 1], A.shape))
    P = ClompParams(inner_steps=32, lr_rel=0.05)
    a = clomp_fp64(Ab, y, 40, P, A_refine=A)
    b = clomp_gram_fp64(Ab, y, 40, P, A_refine=A)
    assert b.support == a.support
    np.testing.assert_allclose(b.x, a.x, rtol=0, atol=1e-10 * np.abs(a.x).max())


def test_gram_clomp_matches_autograd_and_torch_adam_rendering():
    """The Gram-form oracle against the framework rendering (autograd through
    A (mask * s), torch.optim.Adam with the per-iteration learning rate)."""
    torch = pytest.importorskip("torch")
    A, y, _, _ = gaussian_instance(60, 24, 96, 5)
    y = y + 0.01 * np.random.default_rng(60).standard_normal(24)
    P = ClompParams(inner_steps=16, lr_rel=0.05)
    ref = clomp_gram_fp64(A, y, 6, P)
    At, yt = torch.tensor(A), torch.tensor(y)
    s = torch.zeros(96, dtype=torch.float64, requires_grad=True)
    mask = torch.zeros(96, dtype=torch.float64)
    opt, S = None, []
    for t in range(6):
        with torch.no_grad():
            c = At.T @ (yt - At @ (mask * s))
            score = c.abs().clone()
            score[mask.bool()] = -float("inf")
            j = int(torch.argmax(score))
            if t == 0:
                sig = float(c.abs().max())
                opt = torch.optim.Adam([s], lr=1.0, betas=(0.9, 0.999), eps=1e-8 * sig,
                                       foreach=False)
            opt.param_groups[0]["lr"] = 0.05 * abs(float(c[j]))
            mask[j] = 1.0
            S.append(j)
        for _ in range(16):
            opt.zero_grad()
            loss = 0.5 * ((At @ (mask * s) - yt) ** 2).sum()
            loss.backward()
            opt.step()
    assert S == ref.support
    np.testing.assert_allclose(s.detach().numpy()[S], ref.extra["s_adam"], rtol=1e-11, atol=1e-13)


def test_incremental_renderings_zero_y_and_capped_k():
    A, _, _, _ = gaussian_instance(61, 6, 20, 2)
    for f in (lambda yy, kk: omp_cgs2_fp64(A, yy, kk),
              lambda yy, kk: clomp_gram_fp64(A, yy, kk, ClompParams())):
        r = f(np.zeros(6), 3)
        assert r.status & ST_ZERO_Y and r.support == []
        r = f(np.ones(6), 9)
        assert r.status & ST_K_CAPPED and len(r.support) == 6
        assert r.resid_norm < 1e-12      # |S| = m: y is reproduced exactly


def test_separated_prefix_stops_at_first_small_gap_and_disagreement():
    from oracle.omp import SolveResult
    base = SolveResult([5, 1, 9, 3], np.zeros(10), 0.0, [0.5, 0.2, 1e-6, 0.3], [])
    assert separated_prefix(base, [], 1e-4) == 2
    assert separated_prefix(base, [], 1e-7) == 4
    p = SolveResult([5, 2, 9, 3], np.zeros(10), 0.0, [], [])
    assert separated_prefix(base, [p], 1e-7) == 1
    assert common_prefix([1, 2, 3], [1, 2, 3]) == 3 and common_prefix([], [1]) == 0


def test_separation_report_agrees_with_well_separated():
    for seed in range(6):
        A, y, _, _ = gaussian_instance(70 + seed, 48, 160, 6)
        ok1, base = well_separated(A, y, 6, delta=1e-3, u=2.0 ** -8)
        ok2, pre, _ = separation_report(A, y, 6, delta=1e-3, u=2.0 ** -8, base=base)
        assert ok1 == ok2 and (pre == 6) == ok1


def test_perturbed_atoms_relative_size_and_determinism():
    At = np.random.default_rng(1).standard_normal((9000, 7))
    P = perturbed_atoms(At, 2.0 ** -8, 3, chunk=4096)
    np.testing.assert_allclose(np.abs(P / At - 1.0), 2.0 ** -8, rtol=1e-12)
    np.testing.assert_array_equal(P, perturbed_atoms(At, 2.0 ** -8, 3, chunk=4096))
    assert not np.array_equal(P, perturbed_atoms(At, 2.0 ** -8, 4, chunk=4096))
    y = np.arange(1.0, 6.0)
    np.testing.assert_allclose(np.abs(perturbed_vector(y, 2.0 ** -24, 1) / y - 1), 2.0 ** -24,
                               rtol=1e-9)


def test_golden_input_generators_are_deterministic_and_fixed_order():
    specs = W.uneven_specs(4096)
    idx = W.uneven_golden_indices(specs)
    ns = [specs[i].n for i in idx]
    assert len(idx) == 16 == len(set(idx)) and ns == sorted(ns)
    assert max(ns) == max(sp.n for sp in specs)           # includes the largest n
    a = W.uneven_instance_golden(idx[0], specs[idx[0]])
    b = W.uneven_instance_golden(idx[0], specs[idx[0]])
    np.testing.assert_array_equal(a.At, b.At)
    np.testing.assert_array_equal(a.y, b.y)
    assert a.At.shape[1] % 32 == 0 and not a.At[:, a.m:].any()
    y64 = a.A[:, a.support] @ a.s[a.support]
    np.testing.assert_allclose(a.y, y64, rtol=1e-6, atol=1e-6 * np.abs(y64).max())
    v = W.bf16_values(np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5e-3], np.float32))
    np.testing.assert_array_equal(v[:3], [1.0, 1.0, 1.0 + 4 * 2.0 ** -8])   # ties to even
    assert v.dtype == np.float32 and abs(v[3] / -2.5e-3 - 1) <= 2.0 ** -9
