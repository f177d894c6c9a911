"""GPU parity of the shared-dictionary schedule: when every iterated signal
of a batch has the same A, the library forms the full Gram matrix A^T A and
every c0 = A^T y once and iterates without passes over A.  Checked against
the FP64 oracle per column (well-separated columns: support identity, final
x within 1e-5), against the per-signal schedule, with the total-variation
prior, and on a 4K-scale image batch (3840 columns of n = 2160) by sampled
columns.
"""

import numpy as np
import pytest
import torch

from oracle import ClompParams
from paper_2501_11592_amd import clomp as C
from paper_2501_11592_amd import workloads as W
from tests.gpu_helpers import FP32_DELTA, FP32_U, compare, dev, oracle_final_x, PARAMS

pytestmark = pytest.mark.gpu

f32 = lambda v: float(np.float32(v))
ITER = C.FLAG_NO_FUSED_SMALL   # keep the image columns out of the fused loop


def _solve(method, b, flags, rscan_min_t=0, shared_min_tiles=0, **kw):
    sol = C.Solver(0, method=method, flags=flags, **kw)
    if rscan_min_t or shared_min_tiles:
        # shared_min_tiles = 1: IHT and paper mode take the shared schedule even
        # for batches whose contraction has few output tiles
        sol.set_tuning(rscan_min_t=rscan_min_t, shared_min_tiles=shared_min_tiles)
    out = sol.solve_shared(dev(b.At), b.m, dev(b.Y), b.k)
    torch.cuda.synchronize()
    sol.close()
    return out


# the correlation scan: always C = A^T R over the batch's residuals, or
# always c0 - Gf[:, S] s per signal
SCANS = {"atr": 1, "gram": 65536}


@pytest.mark.parametrize("scan", sorted(SCANS))
@pytest.mark.parametrize("method", ["clomp", "omp"])
@pytest.mark.parametrize("sr", [0.3, 0.5])
def test_shared_gram_image_batch(method, sr, scan):
    """256 columns sharing A (m = 77 / 128), iterated: the shared schedule
    (either scan) against the oracle, and the same supports as the per-signal
    schedule on the columns both match the oracle."""
    b = W.image_batch(sr)
    out = _solve(method, b, ITER, rscan_min_t=SCANS[scan])
    ref_sched = _solve(method, b, ITER | C.FLAG_NO_SHARED_GRAM)
    kinds = []
    for c in range(0, 256, 8):
        res = oracle_final_x(method, b.A, b.Y[c], b.k)
        kind = compare(out, c, res, b.A, b.Y[c], delta=FP32_DELTA, u=FP32_U, method=method,
                       A_sel=b.A, k=b.k, tol_x=1e-5)
        kinds.append(kind)
        if kind == "identical":
            assert out.support[c].tolist() == ref_sched.support[c].tolist()
    print(f"{method} sr={sr} {scan}: identical {kinds.count('identical')}/{len(kinds)}")
    assert kinds.count("identical") >= len(kinds) // 2
    assert (out.status.cpu().numpy() == 0).all()


def test_shared_gram_with_prior():
    """The prior's diagonal through the shared Gram diagonal."""
    w = 3.0
    b = W.image_batch(0.3)
    out = _solve("clomp", b, ITER, prior_tv=w)
    prm = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                      eps_rel=f32(1e-8), prior_tv=f32(w))
    kinds = []
    for c in range(0, 256, 16):
        res = oracle_final_x("clomp", b.A, b.Y[c], b.k, params=prm)
        kinds.append(compare(out, c, res, b.A, b.Y[c], delta=FP32_DELTA, u=FP32_U,
                             method="clomp", A_sel=b.A, k=b.k, tol_x=1e-5, sep_params=prm))
    print(f"prior: identical {kinds.count('identical')}/{len(kinds)}")
    assert kinds.count("identical") >= len(kinds) // 2


def test_shared_gram_image4k_sampled():
    """3840 columns of n = 2160, m = 648, k = 108 in one call; eight sampled
    columns against the oracle."""
    b = W.image4k_batch(0.3)
    out = _solve("clomp", b, 0)
    assert (out.n_selected.cpu().numpy() == b.k).all()
    assert (out.status.cpu().numpy() == 0).all()
    kinds = []
    for c in range(0, 3840, 480):
        res = oracle_final_x("clomp", b.A, b.Y[c], b.k)
        kinds.append(compare(out, c, res, b.A, b.Y[c], delta=FP32_DELTA, u=FP32_U,
                             method="clomp", A_sel=b.A, k=b.k, tol_x=1e-5))
    print(f"image4k: identical {kinds.count('identical')}/{len(kinds)}")
    assert kinds.count("identical") >= 4


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_shared_gram_graph_replay(method):
    """The shared-dictionary launch sequence captured into a HIP graph on a
    created stream and replayed (new output buffers each call): every replay
    equals the eager solve bit for bit."""
    b = W.image_batch(0.3)
    At, Y = dev(b.At), dev(b.Y)
    eager = _solve(method, b, ITER)
    sol = C.Solver(0, method=method, flags=ITER | C.FLAG_GRAPH)
    stream = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(stream):
            outs.append(sol.solve_batch([dict(At=At, m=b.m, y=Y[c], k=b.k)
                                         for c in range(Y.shape[0])], stream=stream))
        stream.synchronize()
        torch.cuda.synchronize()   # eager work of the program between replays
    for out in outs:
        for c in range(0, 256, 5):
            assert out.support[c].tolist() == eager.support[c].tolist(), c
            assert torch.equal(out.x[c], eager.x[c]), c
        assert torch.equal(out.resid_norm, eager.resid_norm)
    sol.close()


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_shared_gram_edges(method):
    """A shared A whose lda padding holds NaN, columns with k = 32, 16 and 8
    (signals leave the active prefix at different iterations) and one zero
    column y: the zero column returns x = 0 with the zero-y bit, the others
    match the oracle where well separated."""
    b = W.image_batch(0.3, lda=96)
    At = b.At.copy()
    At[:, b.m:] = np.nan
    Y = b.Y.copy()
    Y[7] = 0.0
    ks = [(32, 16, 8)[c % 3] for c in range(256)]
    sol = C.Solver(0, method=method, flags=ITER)
    At_d, Y_d = dev(At), dev(Y)
    out = sol.solve_batch([dict(At=At_d, m=b.m, y=Y_d[c], k=ks[c]) for c in range(256)])
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert st[7] & C.ST_ZERO_Y and int(out.n_selected[7]) == 0 and not out.x[7].any()
    assert not (st & C.ST_NAN).any()
    for c in range(256):
        if c != 7:
            assert int(out.n_selected[c]) == ks[c], c
    kinds = []
    for c in range(0, 256, 9):
        if c == 7:
            continue
        res = oracle_final_x(method, b.A, Y[c], ks[c])
        kinds.append(compare(out, c, res, b.A, Y[c], delta=FP32_DELTA, u=FP32_U, method=method,
                             A_sel=b.A, k=ks[c], tol_x=1e-5))
    print(f"{method} edges: identical {kinds.count('identical')}/{len(kinds)}")
    assert kinds.count("identical") >= len(kinds) // 2
    sol.close()


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_shared_gram_large_support_teams(method):
    """Four signals sharing A (n=2048, m=1024) with k = 300: supports beyond
    256 atoms run the coefficient teams, reading the Gram row through the
    shared matrix, and the residual by row tiles."""
    g = np.random.default_rng(1777)
    n, m, k = 2048, 1024, 300
    A = g.standard_normal((m, n)) / np.sqrt(m)
    At = np.ascontiguousarray(A.T.astype(np.float32))
    A = At.T.astype(np.float64)
    sigs = []
    for i in range(4):
        x = np.zeros(n)
        x[g.choice(n, k, replace=False)] = g.standard_normal(k)
        sigs.append((A @ x).astype(np.float32))
    At_d = dev(At)
    sol = C.Solver(0, method=method)
    out = sol.solve_batch([dict(At=At_d, m=m, y=dev(y), k=k) for y in sigs])
    torch.cuda.synchronize()
    assert (out.status.cpu().numpy() == 0).all()
    assert (out.n_selected.cpu().numpy() == k).all()
    res = oracle_final_x(method, A, sigs[0].astype(np.float64), k)
    kind = compare(out, 0, res, A, sigs[0].astype(np.float64), delta=FP32_DELTA, u=FP32_U,
                   method=method, A_sel=A, k=k, tol_x=1e-5)
    print(f"{method} k=300 shared: {kind}")
    # the oracle separates the CLOMP solve of this signal, not the OMP one;
    # OMP's x is then checked as the least squares on the GPU's own support
    if method == "clomp":
        assert kind == "identical"
    else:
        from oracle import lstsq_support
        from tests.gpu_helpers import rel_err
        S = out.support[0].cpu().numpy().tolist()
        x = out.x[0].cpu().numpy().astype(np.float64)
        assert rel_err(x[S], lstsq_support(A, sigs[0].astype(np.float64), S)) <= 1e-5
    sol.close()


@pytest.mark.parametrize("method", ["iht", "clomp_paper"])
def test_shared_gradient_iht_and_paper_mode(method):
    """IHT and paper mode on 256 columns sharing A: the gradient of each
    iteration is one contraction A^T R for the batch.  Against the oracle on
    well-separated columns and against the per-signal scan (supports equal
    where the oracle asserts them)."""
    from oracle import iht_fp64, clomp_paper_fp64, PaperParams, well_separated
    from tests.gpu_helpers import rel_err
    R = 20
    b = W.image_batch(0.3)
    out = _solve(method, b, 0, inner_steps=R, shared_min_tiles=1)
    per = _solve(method, b, C.FLAG_NO_SHARED_GRAM, inner_steps=R)
    prm = PaperParams(threshold=f32(0.7), max_iters=R, lr_rel=f32(0.05), beta1=f32(0.9),
                      beta2=f32(0.999), eps_rel=f32(1e-8))
    ident = total = 0
    for c in range(0, 256, 8):
        y = b.Y[c].astype(np.float64)
        if method == "iht":
            ref = iht_fp64(b.A, y, b.k, max_iters=R)
            from types import SimpleNamespace
            sep = SimpleNamespace(max_iters=R)
        else:
            ref = clomp_paper_fp64(b.A, y, b.k, prm)
            sep = prm
        ok, _ = well_separated(b.A, y, b.k, method=method, params=sep, delta=FP32_DELTA,
                               u=FP32_U, base=ref)
        total += 1
        if not ok:
            continue
        supp = out.support[c][:int(out.n_selected[c])].tolist()
        assert supp == ref.support, (c, supp, ref.support)
        assert supp == per.support[c][:int(per.n_selected[c])].tolist(), c
        assert rel_err(out.x[c].cpu().numpy().astype(np.float64), ref.x) <= 1e-5, c
        ident += 1
    print(f"{method} shared gradient: identical {ident}/{total}")
    assert ident >= total // 3


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_shared_gram_bf16_with_master(method):
    """BF16 bulk with an FP32 master on a shared dictionary (n=512, m=128, 64
    signals of 10 Gaussian non-zeros): the full Gram matrix, c0 and the A^T R
    scan contract the BF16 values (FP32 accumulation), the refinement uses the
    master.  Against the oracle run on the BF16 values (selection) and the
    master (refinement); the BF16 separation criterion holds for about two
    thirds of such signals."""
    from tests.gpu_helpers import BF16_DELTA, BF16_U
    g = np.random.default_rng(2024)
    n, m, k, a = 512, 128, 10, 64
    A32 = (g.standard_normal((m, n)) / np.sqrt(m)).astype(np.float32)
    At = np.ascontiguousarray(A32.T)
    A = A32.astype(np.float64)
    Abf = torch.from_numpy(A32).to(torch.bfloat16).to(torch.float64).numpy()
    ys = []
    for _ in range(a):
        x = np.zeros(n)
        x[g.choice(n, k, replace=False)] = g.standard_normal(k)
        ys.append((A @ x).astype(np.float32))
    At32 = dev(At)
    Atb = At32.to(torch.bfloat16)
    sol = C.Solver(0, method=method, flags=ITER)
    out = sol.solve_batch([dict(At=Atb, At_master=At32, m=m, y=dev(y), k=k) for y in ys])
    torch.cuda.synchronize()
    assert (out.status.cpu().numpy() == 0).all()
    kinds = []
    for c in range(0, a, 4):
        y = ys[c].astype(np.float64)
        res = oracle_final_x(method, Abf, y, k, A_refine=A)
        kinds.append(compare(out, c, res, A, y, delta=BF16_DELTA, u=BF16_U, method=method,
                             A_sel=Abf, k=k, tol_x=1e-3))
    print(f"{method} bf16 shared: identical {kinds.count('identical')}/{len(kinds)}")
    assert kinds.count("identical") >= len(kinds) // 3
    sol.close()


@pytest.mark.parametrize("method", ["clomp", "omp", "iht"])
def test_shared_ragged_tiles_nan_padding(method):
    """Ragged contraction tiles on both sides (n = 300 atoms, 200 columns:
    neither a multiple of 128) with m = 77 (a partial group of four k) and
    NaN in every lda padding entry: every mode of the shared contraction
    (A^T A, A^T Y, the scan or the IHT gradient) must mask the padding and the
    rows and columns past the matrix.  No NaN status; supports and x against
    the oracle where well separated and against the per-signal schedule."""
    from oracle import iht_fp64, well_separated
    from tests.gpu_helpers import rel_err
    b = W.image_batch(0.3, n=300, a=200, k=24, lda=96)
    b.At = b.At.copy()
    b.At[:, b.m:] = np.nan   # b.A reads the first m entries of each row only
    R = 20
    flags = ITER if method != "iht" else 0
    kw = {} if method != "iht" else dict(inner_steps=R)
    out = _solve(method, b, flags, shared_min_tiles=1, **kw)
    per = _solve(method, b, flags | C.FLAG_NO_SHARED_GRAM, **kw)
    st = out.status.cpu().numpy()
    assert not (st & C.ST_NAN).any()
    assert all(int(out.n_selected[c]) == b.k for c in range(200))
    ident = total = 0
    for c in range(0, 200, 7):
        y = b.Y[c].astype(np.float64)
        if method == "iht":
            from types import SimpleNamespace
            ref = iht_fp64(b.A, y, b.k, max_iters=R)
            ok, _ = well_separated(b.A, y, b.k, method="iht", params=SimpleNamespace(max_iters=R),
                                   delta=FP32_DELTA, u=FP32_U, base=ref)
            total += 1
            if not ok:
                continue
            supp = out.support[c][:int(out.n_selected[c])].tolist()
            assert supp == ref.support, (c, supp, ref.support)
            assert rel_err(out.x[c].cpu().numpy().astype(np.float64), ref.x) <= 1e-5, c
            kind = "identical"
        else:
            res = oracle_final_x(method, b.A, b.Y[c], b.k)
            kind = compare(out, c, res, b.A, b.Y[c], delta=FP32_DELTA, u=FP32_U, method=method,
                           A_sel=b.A, k=b.k, tol_x=1e-5)
            total += 1
        if kind == "identical":
            ident += 1
            assert out.support[c].tolist() == per.support[c].tolist(), c
    print(f"{method} ragged shared tiles: identical {ident}/{total}")
    assert ident >= total // 3


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_shared_bf16_ragged_tiles_nan_padding(method):
    """BF16 bulk on a shared dictionary with ragged contraction tiles (n = 300
    atoms, 200 columns), m = 77 (a partial chunk of k) and a NaN in every lda
    padding entry of the BF16 matrix: the BF16 matrix-core Gram matrix and
    scan (residuals rounded to BF16) must mask the padding.  No NaN status;
    on every sampled column the ordered support equals the oracle's (on the
    BF16 values, refinement on the FP32 master) over its separated prefix
    under the BF16 gates, and x is the least squares on the GPU's support."""
    from oracle import lstsq_support, separation_report
    from tests.gpu_helpers import BF16_DELTA, BF16_U, PARAMS, rel_err
    b = W.image_batch(0.3, n=300, a=200, k=24, lda=96)
    A = b.A                                            # float32 values, float64
    Abf = torch.from_numpy(b.At[:, :b.m]).to(torch.bfloat16).to(torch.float64).numpy().T
    At32 = dev(b.At)
    Atb = torch.zeros((b.n, 128), dtype=torch.bfloat16, device="cuda")
    Atb[:, :b.m] = At32[:, :b.m].to(torch.bfloat16)
    Atb[:, b.m:] = float("nan")
    sol = C.Solver(0, method=method, flags=ITER)
    out = sol.solve_batch([dict(At=Atb, At_master=At32, m=b.m, y=dev(b.Y[c]), k=b.k)
                           for c in range(200)])
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert not (st & C.ST_NAN).any()
    assert all(int(out.n_selected[c]) == b.k for c in range(200))
    total = 0
    for c in range(0, 200, 7):
        y = b.Y[c].astype(np.float64)
        res = oracle_final_x(method, Abf, y, b.k, A_refine=A)
        _, pre, _ = separation_report(Abf, y, b.k, method=method, params=PARAMS,
                                      delta=BF16_DELTA, u=BF16_U, A_refine=A, base=res)
        S = out.support[c].cpu().numpy().tolist()
        assert S[:pre] == res.support[:pre], (c, pre)
        x = out.x[c].cpu().numpy().astype(np.float64)
        assert rel_err(x[S], lstsq_support(A, y, S)) <= 1e-5, c
        total += pre
    print(f"{method} bf16 ragged shared tiles: {total} selections in separated prefixes")
    # the oracle's separated prefixes of the 29 sampled columns hold 317
    # (CLOMP) / 278 (OMP) of their 696 selections
    assert total >= {"clomp": 317, "omp": 278}[method]
    sol.close()
