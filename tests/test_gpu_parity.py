"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Support identity is asserted on well-separated instances (per-iteration gap
and perturbation stability, see oracle.separation); final coefficients within
1e-5 relative (FP32 bulk) or 1e-3 (BF16 bulk with FP32 refinement); the
reported FP64 residual norm is checked against its closed form.
"""

import math

import numpy as np
import pytest
import torch

from oracle import clomp_fp64, omp_fp64
from paper_2501_11592_amd import clomp as C
from paper_2501_11592_amd import workloads as W
from tests.gpu_helpers import (PARAMS, FP32_DELTA, FP32_U, BF16_DELTA, BF16_U, dev,
                               oracle_final_x, compare, rel_err)

pytestmark = pytest.mark.gpu


# the two iterated schedules with the fused small-signal loop off, and the
# default configuration (small signals fused, the rest iterated)
FLOWS = {"resid": C.FLAG_RESIDUAL_FLOW | C.FLAG_NO_FUSED_SMALL,
         "corr": C.FLAG_CORR_FLOW | C.FLAG_NO_FUSED_SMALL,
         "fused": 0}


@pytest.fixture(scope="module", params=sorted(FLOWS))
def solvers(request):
    """CLOMP and OMP handles, under each configuration."""
    fl = FLOWS[request.param]
    s = {"clomp": C.Solver(0, method="clomp", flags=fl),
         "omp": C.Solver(0, method="omp", flags=fl)}
    yield s
    for v in s.values():
        v.close()


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


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_small_single_signals(solvers, method):
    """n=256, m=64, k=8: twenty signals in one batch."""
    sigs = [W.single_small(i) for i in range(20)]
    out = solvers[method].solve_batch(_items(sigs))
    torch.cuda.synchronize()
    kinds = []
    for i, s in enumerate(sigs):
        res = oracle_final_x(method, s.A, s.y, s.k)
        kinds.append(compare(out, i, res, s.A, s.y, delta=FP32_DELTA, u=FP32_U, method=method,
                             A_sel=s.A, k=s.k, tol_x=1e-5))
        assert int(out.status[i]) == 0
        assert int(out.n_selected[i]) == 8
    assert kinds.count("identical") >= 15, kinds


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_ragged_sizes_span_tiles(solvers, method):
    """Sizes that are not multiples of the vector width or tile, with lda
    padding filled with NaN (the kernels must ignore entries beyond m)."""
    rng = np.random.default_rng(5)
    sigs = []
    for i, (n, m, k) in enumerate([(1000, 77, 9), (3001, 130, 12), (517, 26, 26), (700, 299, 31)]):
        s = W.single_small(100 + i, n=n, m=m, k=k)
        At = s.At.copy()
        At[:, m:] = np.nan
        s.At = At
        sigs.append(s)
    out = solvers[method].solve_batch(_items(sigs))
    torch.cuda.synchronize()
    ident = 0
    for i, s in enumerate(sigs):
        res = oracle_final_x(method, s.A, s.y, s.k)
        ident += compare(out, i, res, s.A, s.y, delta=FP32_DELTA, u=FP32_U, method=method,
                         A_sel=s.A, k=s.k, tol_x=1e-5) == "identical"
        assert not (int(out.status[i]) & C.ST_NAN)
    assert ident >= 2


@pytest.mark.parametrize("sr", [0.1, 0.3, 0.5])
def test_image_batch_shared_matrix(solvers, sr):
    """256 columns of a synthetic image sharing one Gaussian A (m = 26/77/128),
    solved in one call; a subset of columns is checked against the oracle."""
    b = W.image_batch(sr)
    At = dev(b.At)
    Y = dev(b.Y)
    out = solvers["clomp"].solve_shared(At, b.m, Y, b.k)
    torch.cuda.synchronize()
    k_eff = min(b.k, b.m)
    assert (out.n_selected.cpu().numpy() == k_eff).all()
    capped = (out.status.cpu().numpy() & C.ST_K_CAPPED) != 0
    assert capped.all() == (b.k > b.m)
    kinds = []
    for c in range(0, 256, 16):
        res = oracle_final_x("clomp", b.A, b.Y[c], b.k)
        kinds.append(compare(out, c, res, b.A, b.Y[c], delta=FP32_DELTA, u=FP32_U,
                             method="clomp", A_sel=b.A, k=b.k,
                             tol_x=1e-5 if sr > 0.1 else 1e-3))
    print(f"sr={sr}: identical {kinds.count('identical')}/{len(kinds)}")
    # compare() asserts every column the oracle calls well separated; the
    # oracle separates 15 / 16 / 16 of these 16 columns
    assert kinds.count("identical") == {0.1: 15, 0.3: 16, 0.5: 16}[sr]


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_uneven_bf16_batch_with_master(solvers, method):
    """Uneven batch, BF16 bulk with FP32 master (selection on the BF16 values,
    refinement on the master)."""
    specs = [sp for sp in W.uneven_specs(400) if sp.n <= 1400][:24]
    sigs = [W.uneven_instance_host(i, sp) for i, sp in enumerate(specs)]
    out = solvers[method].solve_batch(_items(sigs, torch.bfloat16))
    torch.cuda.synchronize()
    ident = 0
    for i, s in enumerate(sigs):
        Abf = torch.from_numpy(s.At[:, :s.m]).to(torch.bfloat16).to(torch.float64).numpy().T
        res = oracle_final_x(method, Abf, s.y, s.k, A_refine=s.A)
        kind = compare(out, i, res, s.A, s.y, delta=BF16_DELTA, u=BF16_U, method=method,
                       A_sel=Abf, k=s.k, tol_x=1e-3)
        ident += kind == "identical"
        assert int(out.n_selected[i]) == min(s.k, s.m, s.n)
    print(f"{method}: identical {ident}/{len(sigs)}")
    # compare() asserts every instance the oracle calls well separated: 7 of
    # the 24 for CLOMP, 3 for OMP under the BF16 gates
    assert ident == {"clomp": 7, "omp": 3}[method]


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_coefficient_teams(method):
    """Correlation-update schedule with the coefficient update split over a
    team of workgroups once the support exceeds 16 atoms (team_min_rows = 16):
    up to ceil(80 / 16) = 5 members per signal, four signals per launch.
    Checked against the oracle and against the single-workgroup update."""
    sigs = [W.single_small(200 + i, n=2048, m=384, k=80) for i in range(4)]
    team = C.Solver(0, method=method, flags=C.FLAG_CORR_FLOW)
    team.set_tuning(team_min_rows=16)
    assert team.get_tuning()["team_min_rows"] == 16
    single = C.Solver(0, method=method, flags=C.FLAG_CORR_FLOW)
    out = team.solve_batch(_items(sigs))
    out1 = single.solve_batch(_items(sigs))
    torch.cuda.synchronize()
    ident = 0
    for i, s in enumerate(sigs):
        assert int(out.status[i]) == 0 and int(out.n_selected[i]) == s.k
        res = oracle_final_x(method, s.A, s.y, s.k)
        kind = compare(out, i, res, s.A, s.y, delta=FP32_DELTA, u=FP32_U, method=method,
                       A_sel=s.A, k=s.k, tol_x=1e-5)
        if kind == "identical":
            ident += 1
            assert out1.support[i].tolist() == out.support[i].tolist()
            assert rel_err(out.x[i].cpu().numpy().astype(np.float64),
                           out1.x[i].cpu().numpy().astype(np.float64)) <= 1e-5
    print(f"{method} teams: identical {ident}/{len(sigs)}")
    assert ident >= 2
    team.close()
    single.close()


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_team_watchdog_forced_from_host(method):
    """The bounded team wait, forced to give up from the host: a spin limit of
    one poll per wait.  Some signal must carry CLOMP_ST_WATCHDOG, every kernel
    must still finish (the device synchronises without error), and with the
    default limit restored the same handle solves exactly as a fresh one."""
    sigs = [W.single_small(200 + i, n=2048, m=384, k=80) for i in range(4)]
    items = _items(sigs)
    team = C.Solver(0, method=method, flags=C.FLAG_CORR_FLOW)
    team.set_tuning(team_min_rows=16, spin_limit=1)
    assert team.get_tuning()["spin_limit"] == 1
    out = team.solve_batch(items)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    print(f"{method}: status bits with spin_limit 1: {st.tolist()}")
    assert (st & C.ST_WATCHDOG).any()
    assert ((st & ~(C.ST_WATCHDOG | C.ST_REFINE_INACCURATE)) == 0).all()
    team.set_tuning(spin_limit=-1)
    assert team.get_tuning()["spin_limit"] == 1 << 20
    again = team.solve_batch(items)
    fresh = C.Solver(0, method=method, flags=C.FLAG_CORR_FLOW)
    fresh.set_tuning(team_min_rows=16)
    ref = fresh.solve_batch(items)
    torch.cuda.synchronize()
    assert (again.status.cpu().numpy() == 0).all()
    for i in range(len(sigs)):
        assert torch.equal(again.support[i], ref.support[i])
        assert torch.equal(again.x[i], ref.x[i])
    team.close()
    fresh.close()


@pytest.mark.parametrize("flow", ["resid", "corr"])
def test_autotune_matches_default(flow):
    """CLOMP_FLAG_AUTOTUNE times the candidate tile sizes on the first call of a
    size class and reuses the choice; tiles only regroup atoms across
    workgroups, so the results are bit-identical to the default tiles."""
    sigs = [W.single_small(300 + i, n=3000, m=200, k=20) for i in range(3)]
    fl = FLOWS[flow]
    tuned = C.Solver(0, method="clomp", flags=fl | C.FLAG_AUTOTUNE)
    plain = C.Solver(0, method="clomp", flags=fl)
    a = tuned.solve_batch(_items(sigs))
    b = plain.solve_batch(_items(sigs))
    a2 = tuned.solve_batch(_items(sigs))
    torch.cuda.synchronize()
    kb = tuned.get_tuning()
    if flow == "corr":
        assert kb["pass_tile_kb"] in (128, 256, 512, 1024, 2048)
    else:
        assert kb["scan_tile_kb"] in (32, 64, 128, 256, 512)
    print(f"{flow}: tuned {kb}")
    for i in range(len(sigs)):
        assert torch.equal(a.support[i], b.support[i]) and torch.equal(a2.support[i], b.support[i])
        assert torch.equal(a.x[i], b.x[i]) and torch.equal(a2.x[i], b.x[i])
    tuned.close()
    plain.close()


def test_prepared_batch_reruns(solvers):
    """Descriptors packed once: repeated launches rewrite the same outputs with
    the results of a one-off solve."""
    sigs = [W.single_small(400 + i) for i in range(5)] + [W.single_small(410, n=2000, m=150, k=30)]
    sol = solvers["clomp"]
    stream = torch.cuda.Stream()
    prep = sol.prepare(_items(sigs), stream=stream)
    r1 = sol.run(prep)
    torch.cuda.synchronize()
    x1 = [t.clone() for t in r1.x]
    r2 = sol.run(prep)
    ref = sol.solve_batch(_items(sigs))
    torch.cuda.synchronize()
    assert r2 is r1
    for i in range(len(sigs)):
        assert torch.equal(r2.x[i], x1[i]) and torch.equal(r2.x[i], ref.x[i])
        assert torch.equal(r2.support[i], ref.support[i])


def test_plan_reuse_with_new_pointers(solvers):
    """A batch with the shapes of the previous call reuses its plan with the
    new data pointers: results equal those of a fresh handle."""
    mk = lambda base: [W.single_small(base + i) for i in range(4)] + \
        [W.single_small(base + 9, n=1500, m=120, k=24)]
    sol = solvers["omp"]
    sol.solve_batch(_items(mk(500)))
    b = sol.solve_batch(_items(mk(600)))
    fresh = C.Solver(0, method="omp", flags=sol.params.flags)
    ref = fresh.solve_batch(_items(mk(600)))
    torch.cuda.synchronize()
    for i in range(5):
        assert torch.equal(b.support[i], ref.support[i])
        assert torch.equal(b.x[i], ref.x[i])
    fresh.close()


def test_large_support_single_workgroup():
    """k = 300 under the correlation-update schedule with coefficient teams
    off: iterations with 256 < t+1 <= 300 run the split-row Adam of a single
    1024-thread workgroup, reading G from memory."""
    s = W.single_small(700, n=2048, m=1024, k=300)
    sol = C.Solver(0, method="clomp", flags=C.FLAG_CORR_FLOW | C.FLAG_NO_FUSED_SMALL)
    sol.set_tuning(team_min_rows=65536)
    out = sol.solve_batch(_items([s]))
    torch.cuda.synchronize()
    assert int(out.status[0]) == 0 and int(out.n_selected[0]) == 300
    res = oracle_final_x("clomp", s.A, s.y, s.k)
    kind = compare(out, 0, res, s.A, s.y, delta=FP32_DELTA, u=FP32_U, method="clomp",
                   A_sel=s.A, k=s.k, tol_x=1e-5)
    assert kind == "identical"    # the oracle calls this instance well separated
    sol.close()


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_many_iterated_signals_split_launch(method):
    """More active signals than CUs under the correlation-update schedule: the
    CLOMP coefficient update runs in support-sized workgroups and the pass in
    a launch of its own (OMP keeps the fused launch).  600 distinct small signals (n=256, m=64, k=8, and
    k=24 for every fifth) kept out of the fused loop; every fifteenth against
    the oracle, the rest against the fused path's supports."""
    sigs = [W.single_small(1600 + i, k=24 if i % 5 == 0 else 8) for i in range(600)]
    items = _items(sigs)
    sol = C.Solver(0, method=method, flags=C.FLAG_CORR_FLOW | C.FLAG_NO_FUSED_SMALL)
    out = sol.solve_batch(items)
    fused = C.Solver(0, method=method)
    ref = fused.solve_batch(items)
    torch.cuda.synchronize()
    assert (out.status.cpu().numpy() == 0).all()
    kinds = []
    for i in range(0, 600, 15):
        res = oracle_final_x(method, sigs[i].A, sigs[i].y, sigs[i].k)
        kinds.append(compare(out, i, res, sigs[i].A, sigs[i].y, delta=FP32_DELTA, u=FP32_U,
                             method=method, A_sel=sigs[i].A, k=sigs[i].k, tol_x=1e-5))
    print(f"{method} split launch: identical {kinds.count('identical')}/{len(kinds)}")
    assert kinds.count("identical") >= len(kinds) * 3 // 4
    same = sum(out.support[i].tolist() == ref.support[i].tolist() for i in range(600))
    assert same >= 570, same
    sol.close()
    fused.close()


def test_edge_cases(solvers):
    sol = solvers["clomp"]
    base = W.single_small(7)
    # y == 0 -> empty support, x = 0, ZERO_Y
    zero = W.single_small(7)
    zero.y = np.zeros_like(zero.y)
    # k > m -> capped at m (square system)
    cap = W.single_small(8, n=40, m=12, k=30)
    # n == k_eff == m, tiny
    tiny = W.single_small(9, n=5, m=5, k=5)
    # duplicate columns: tie broken to the lower index
    dup = W.single_small(10, n=64, m=32, k=1)
    dup.At[40] = dup.At[3]
    dup.y = (dup.At[3, :32].astype(np.float64) * 2.0 + dup.At[10, :32] * 0.5).astype(np.float32)
    sigs = [base, zero, cap, tiny, dup]
    out = sol.solve_batch(_items(sigs))
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert st[0] == 0
    assert st[1] & C.ST_ZERO_Y and int(out.n_selected[1]) == 0
    assert not out.x[1].any() and float(out.resid_norm[1]) == 0.0
    assert (out.support[1].cpu().numpy() == -1).all()
    assert st[2] & C.ST_K_CAPPED and int(out.n_selected[2]) == 12
    assert int(out.n_selected[3]) == 5
    assert float(out.resid_norm[3]) < 1e-4 * np.linalg.norm(tiny.y)
    assert int(out.support[4][0]) == 3    # |c_3| == |c_40|: lowest index wins
    # tiny with k_eff = m: the full square system is solved exactly
    res = clomp_fp64(tiny.A, tiny.y, 5, PARAMS)
    assert sorted(out.support[3].cpu().numpy().tolist()) == sorted(res.support)


def test_deterministic(solvers):
    sigs = [W.single_small(i) for i in range(6)] + [W.single_small(50, n=3000, m=200, k=40)]
    a = solvers["clomp"].solve_batch(_items(sigs))
    torch.cuda.synchronize()
    xa = [t.clone() for t in a.x]
    b = solvers["clomp"].solve_batch(_items(sigs))
    torch.cuda.synchronize()
    for u, v in zip(xa, b.x):
        assert torch.equal(u, v)
    assert torch.equal(a.resid_norm, b.resid_norm)


def test_grad_fp32_against_oracle(solvers):
    from oracle import grad_fp64
    s = W.single_small(3, n=300, m=70, k=10)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(300).astype(np.float32)
    mask = (rng.random(300) < 0.3).astype(np.uint8)
    loss, gx, u = solvers["clomp"].grad(dev(s.At), s.m, dev(x), dev(mask), dev(s.y))
    torch.cuda.synchronize()
    l64, g64, u64 = grad_fp64(x, mask, s.A, s.y)
    # normwise FP32 bound: 10 * sqrt(m) * 2^-24 * ||A|| * (||A(mask x)|| + ||y||)
    bound = 10 * math.sqrt(s.m) * 2.0 ** -24 * np.linalg.norm(s.A, 2) * (
        np.linalg.norm(s.A @ (mask * x.astype(np.float64))) + np.linalg.norm(s.y))
    assert np.max(np.abs(gx.cpu().numpy() - g64)) <= bound * np.linalg.norm(s.A, 2)
    assert np.max(np.abs(u.cpu().numpy() - u64)) <= bound
    assert abs(float(loss) - l64) <= 1e-5 * max(1.0, l64)
    assert not gx.cpu().numpy()[mask == 0].any()


def test_grad_fp64_gradcheck_and_autograd(solvers):
    s = W.single_small(4, n=40, m=16, k=4, dtype=np.float64)
    At = dev(s.At)
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.standard_normal(40), device="cuda", requires_grad=True)
    y = torch.tensor(s.y.astype(np.float64), device="cuda", requires_grad=True)
    mask = dev((rng.random(40) < 0.5).astype(np.uint8))
    f = lambda xx, yy: C.ClompLoss.apply(xx, mask, At, s.m, yy)
    assert torch.autograd.gradcheck(f, (x, y), eps=1e-6, atol=1e-8, rtol=1e-6)
    # central differences on the FP64 HIP path are exact for the quadratic loss
    from oracle import grad_fp64
    l64, g64, _ = grad_fp64(x.detach().cpu().numpy(), mask.cpu().numpy(), s.A, s.y)
    loss = f(x, y)
    loss.backward()
    np.testing.assert_allclose(x.grad.cpu().numpy(), g64, rtol=1e-12, atol=1e-12)
    assert abs(loss.item() - l64) <= 1e-12 * max(1, l64)


def test_grad_fp64_gradcheck_uneven_instances():
    """FP64 gradcheck of the hand-written backward on the eight smallest
    instances of the uneven batch's size distribution (n log-uniform in
    [512, 8192], m/n in [0.1, 0.5], k in [n/64, n/16]): A iid N(0, 1/m), mask
    on k random atoms, random x and y; and the gradient against the oracle's
    to 1e-12."""
    from oracle import grad_fp64
    specs = W.uneven_specs(4096)
    order = np.argsort([sp.n for sp in specs], kind="stable")[:8]
    for i in order:
        sp = specs[i]
        g = np.random.default_rng([2501, 11592, 4, int(i), 9])
        A = g.standard_normal((sp.m, sp.n)) / math.sqrt(sp.m)
        lda = W.pad_lda(sp.m, 8)
        At_h = np.zeros((sp.n, lda))
        At_h[:, :sp.m] = A.T
        mask_h = np.zeros(sp.n, np.uint8)
        mask_h[g.choice(sp.n, sp.k, replace=False)] = 1
        x_h, y_h = g.standard_normal(sp.n), g.standard_normal(sp.m)
        At = dev(At_h)
        mask = dev(mask_h)
        x = dev(x_h).requires_grad_(True)
        y = dev(y_h).requires_grad_(True)
        print(f"gradcheck: uneven instance {i} n={sp.n} m={sp.m} k={sp.k}", flush=True)
        f = lambda xx, yy: C.ClompLoss.apply(xx, mask, At, sp.m, yy)
        assert torch.autograd.gradcheck(f, (x, y), eps=1e-6, atol=1e-8, rtol=1e-6)
        l64, g64, u64 = grad_fp64(x_h, mask_h, A, y_h)
        loss = f(x, y)
        loss.backward()
        np.testing.assert_allclose(x.grad.cpu().numpy(), g64, rtol=1e-12,
                                   atol=1e-12 * np.abs(g64).max())
        np.testing.assert_allclose(y.grad.cpu().numpy(), -u64, rtol=1e-12,
                                   atol=1e-12 * np.abs(u64).max())
        assert abs(loss.item() - l64) <= 1e-12 * l64


def test_abi_errors_on_device(solvers):
    sol = solvers["clomp"]
    s = W.single_small(1)
    it = _items([s])[0]
    it["At"] = torch.zeros((256, 66), device="cuda")   # lda = 66: not a multiple of 4
    with pytest.raises(C.ClompError, match="INVALID_ARGUMENT"):
        sol.solve_batch([it])
    it = _items([s], torch.bfloat16)[0]
    it.pop("At_master")
    # refused by the binding before any launch (the library refuses it too:
    # clomp_check_batch, CPU suite)
    with pytest.raises(C.ClompError, match="float32 At_master"):
        sol.solve_batch([it])
