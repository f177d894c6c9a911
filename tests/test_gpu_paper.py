"""GPU parity of paper-mode CLOMP (normalised-threshold multi-selection, one
Adam step per iteration) against the FP64 oracle.

Support identity is asserted on well-separated instances: in every iteration
the unselected scores |c_j| / max|c| keep a relative distance of at least
delta from the threshold, and the oracle's support is unchanged under relative
perturbations of A and y (oracle.separation); final coefficients (least
squares on the support) within 1e-5 relative (FP32 bulk) or 1e-3 (BF16 bulk
with FP32 master).  Both sides take the same float32 hyper-parameters.
"""

import numpy as np
import pytest
import torch

from oracle import PaperParams, clomp_paper_fp64, well_separated
from paper_2501_11592_amd import clomp as C
from paper_2501_11592_amd import workloads as W
from tests.gpu_helpers import FP32_DELTA, FP32_U, BF16_DELTA, BF16_U, dev, rel_err, fp64_resid

pytestmark = pytest.mark.gpu

f32 = lambda v: float(np.float32(v))


def _params(R, thr=0.7):
    return PaperParams(threshold=f32(thr), max_iters=R, lr_rel=f32(0.05), beta1=f32(0.9),
                       beta2=f32(0.999), eps_rel=f32(1e-8))


def _items(sigs, dtype=torch.float32):
    items = []
    for s in sigs:
        At = dev(s.At)
        it = dict(At=At if dtype == torch.float32 else At.to(torch.bfloat16), m=s.m,
                  y=dev(s.y), k=s.k)
        if dtype != torch.float32:
            it["At_master"] = At
        items.append(it)
    return items


SEEN = C.ST_NAN | C.ST_K_CAPPED | C.ST_ZERO_Y


def _check(out, i, A_sel, A_ref, y, k, prm, delta, u, tol_x):
    """Returns True when the instance is well separated (and then asserted)."""
    nsel = int(out.n_selected[i])
    supp = out.support[i][:nsel].cpu().numpy().tolist()
    x = out.x[i].cpu().numpy().astype(np.float64)
    assert abs(float(out.resid_norm[i]) - fp64_resid(A_ref, y, supp, x)) <= 1e-9 * (
        1 + np.linalg.norm(y))
    assert supp == sorted(supp)                     # index order
    ref = clomp_paper_fp64(A_sel, y, k, prm, A_refine=None if A_sel is A_ref else A_ref)
    ok, _ = well_separated(A_sel, y, k, method="clomp_paper", params=prm, delta=delta, u=u,
                           A_refine=None if A_sel is A_ref else A_ref, base=ref)
    if not ok:
        return False
    assert supp == ref.support, (i, supp, ref.support)
    assert int(out.status[i]) & SEEN == ref.status & SEEN, (i, int(out.status[i]), ref.status)
    assert rel_err(x, ref.x) <= tol_x, (i, rel_err(x, ref.x))
    return True


@pytest.mark.parametrize("R", [1, 5, 200])
def test_paper_small_batch(R):
    """n=256, m=64, k=8: twenty signals in one batch, R iterations, graph
    capture and replay."""
    sigs = [W.single_small(1200 + i) for i in range(20)]
    sol = C.Solver(0, method="clomp_paper", inner_steps=R, flags=C.FLAG_GRAPH)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        out = sol.solve_batch(_items(sigs), stream=stream)
        out = sol.solve_batch(_items(sigs), stream=stream)   # graph replay
    torch.cuda.synchronize()
    prm = _params(R)
    ident = sum(_check(out, i, s.A, s.A, s.y, s.k, prm, FP32_DELTA, FP32_U, 1e-5)
                for i, s in enumerate(sigs))
    print(f"R={R}: identical {ident}/20")
    # the separated set is the oracle's alone (20, 20 and 11 of 20 for
    # R = 1, 5, 200): over 200 iterations some scores pass near T_h
    assert ident >= (10 if R == 200 else 18)
    sol.close()


def test_paper_ragged_sizes_nan_padding():
    """Sizes that are not multiples of the vector width or tile, across lane
    classes and both select widths, with lda padding filled with NaN."""
    sigs = []
    for i, (n, m, k) in enumerate([(1000, 77, 9), (5001, 130, 40), (517, 26, 6), (700, 299, 31)]):
        s = W.single_small(1250 + i, n=n, m=m, k=k)
        At = s.At.copy()
        At[:, m:] = np.nan
        s.At = At
        sigs.append(s)
    sol = C.Solver(0, method="clomp_paper", inner_steps=60)
    out = sol.solve_batch(_items(sigs))
    torch.cuda.synchronize()
    prm = _params(60)
    ident = sum(_check(out, i, s.A, s.A, s.y, s.k, prm, FP32_DELTA, FP32_U, 1e-5)
                for i, s in enumerate(sigs))
    assert not (out.status.cpu().numpy() & C.ST_NAN).any()
    print(f"ragged: identical {ident}/4")
    assert ident >= 2
    sol.close()


def test_paper_bf16_with_master():
    """BF16 bulk with an FP32 master, R = 3: the BF16 separation criterion
    (gap 1e-2, perturbation 2^-8) holds for 7 of the 12 signals at R = 3 and
    for none at R = 20 (multi-selection keeps many scores near T_h)."""
    specs = [sp for sp in W.uneven_specs(400) if sp.n <= 1400][:12]
    sigs = [W.uneven_instance_host(i, sp) for i, sp in enumerate(specs)]
    sol = C.Solver(0, method="clomp_paper", inner_steps=3)
    out = sol.solve_batch(_items(sigs, torch.bfloat16))
    torch.cuda.synchronize()
    prm = _params(3)
    ident = 0
    for i, s in enumerate(sigs):
        Abf = torch.from_numpy(s.At[:, :s.m]).to(torch.bfloat16).to(torch.float64).numpy().T
        ident += _check(out, i, Abf, s.A, s.y, s.k, prm, BF16_DELTA, BF16_U, 1e-3)
    print(f"bf16: identical {ident}/12")
    assert ident >= 6
    sol.close()


def test_paper_large1d():
    """The headline signal (n=16384, m=4096, k=256, float32, noisy), 200
    iterations at T_h = 0.7, against the oracle."""
    sig = W.single_large(0)
    sol = C.Solver(0, method="clomp_paper")
    out = sol.solve_batch([dict(At=dev(sig.At), m=sig.m, y=dev(sig.y), k=sig.k)])
    torch.cuda.synchronize()
    A = sig.A
    y = sig.y.astype(np.float64)
    ok = _check(out, 0, A, A, y, sig.k, _params(200), FP32_DELTA, FP32_U, 1e-5)
    print(f"large1d: separated {ok}, selected {int(out.n_selected[0])}")
    if not ok:
        # not separated: what is unique is checked - the support is a valid
        # paper-mode support and x is the least squares on it (the norm is
        # checked by _check)
        from oracle import lstsq_support
        nsel = int(out.n_selected[0])
        assert 0 < nsel <= sig.k and int(out.status[0]) & C.ST_NAN == 0
        supp = out.support[0][:nsel].cpu().numpy().tolist()
        x = out.x[0].cpu().numpy().astype(np.float64)
        assert rel_err(x[supp], lstsq_support(A, y, supp)) <= 1e-5
    sol.close()


def test_paper_edge_cases_and_determinism():
    """y = 0; k > min(m, n); a first batch larger than k (refused in every
    iteration: empty support, x = 0, ||r|| = ||y||); non-finite y (the loop
    stops with the NaN bit); and two runs bit for bit."""
    base = W.single_small(21)
    zero = W.single_small(22)
    zero.y = np.zeros_like(zero.y)
    cap = W.single_small(23, n=40, m=12, k=30)
    refused = W.single_small(24, k=1)
    nan = W.single_small(25)
    nan.y = nan.y.copy()
    nan.y[3] = np.nan
    sigs = [base, zero, cap, refused, nan]
    sol = C.Solver(0, method="clomp_paper", inner_steps=30, select_threshold=0.05)
    a = sol.solve_batch(_items(sigs))
    torch.cuda.synchronize()
    st = a.status.cpu().numpy()
    prm = _params(30, 0.05)
    for i in (0, 2, 3):
        s = sigs[i]
        ref = clomp_paper_fp64(s.A, s.y, s.k, prm)
        assert int(st[i]) & SEEN == ref.status & SEEN, (i, st[i], ref.status)
    assert st[1] & C.ST_ZERO_Y and int(a.n_selected[1]) == 0 and not a.x[1].any()
    assert st[2] & C.ST_K_CAPPED and int(a.n_selected[2]) <= 12
    assert st[3] & C.ST_K_CAPPED and int(a.n_selected[3]) == 0 and not a.x[3].any()
    assert abs(float(a.resid_norm[3]) - np.linalg.norm(refused.y.astype(np.float64))) <= 1e-6 * (
        np.linalg.norm(refused.y))
    assert st[4] & C.ST_NAN and int(a.n_selected[4]) == 0
    xa = [t.clone() for t in a.x]
    b = sol.solve_batch(_items(sigs))
    torch.cuda.synchronize()
    for u, v in zip(xa, b.x):
        assert torch.equal(u, v)
    sol.close()
