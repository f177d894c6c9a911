"""GPU parity of CLOMP on the columns of one image (CLOMP_FLAG_IMAGE) with the
priors of Eq. (6) (2-D total variation) and Eq. (7) (local variation) against
the FP64 oracle (oracle.image_prior.clomp_image_fp64).

A column is well separated when every one of its iterations has a relative gap
of at least 1e-4 between its two best scores and its support is unchanged when
A and every column of Y are multiplied entrywise by (1 +- 2^-24) (two seeds;
the whole coupled image is re-solved).  There the ordered support must equal
the oracle's and the learned coefficients must agree within 1e-4 relative
(float32 Adam against float64 over k * T coupled steps); everywhere the FP64
residual norm is checked against its closed form on the GPU's own x.
"""

import numpy as np
import pytest
import torch

from oracle import ClompParams, perturbed_atoms, perturbed_vector
from oracle.image_prior import clomp_image_fp64
from paper_2501_11592_amd import clomp as C
from paper_2501_11592_amd import workloads as W
from tests.gpu_helpers import dev, fp64_resid, rel_err

pytestmark = pytest.mark.gpu

f32 = lambda v: float(np.float32(v))
PARAMS = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                     eps_rel=f32(1e-8))


def _separated(A, Y, k, wt, wl, base):
    ok = [bool(r.gaps) and min(r.gaps) >= 1e-4 for r in base]
    for sd in (1, 2):
        Ap = perturbed_atoms(A.T, 2.0 ** -24, sd).T
        Yp = np.stack([perturbed_vector(Y[:, c], 2.0 ** -24, sd + 10 * c)
                       for c in range(Y.shape[1])], axis=1)
        rp = clomp_image_fp64(Ap, Yp, k, PARAMS, w_tv=f32(wt), w_lv=f32(wl))
        ok = [o and rp[c].support == base[c].support for c, o in enumerate(ok)]
    return ok


def _solve(b, wt, wl, flags=C.FLAG_IMAGE, Y=None):
    Y = b.Y if Y is None else Y
    sol = C.Solver(0, method="clomp", flags=flags, prior_tv=wt, prior_lv=wl)
    out = sol.solve_shared(dev(b.At), b.m, dev(Y), b.k)
    torch.cuda.synchronize()
    return sol, out


# the oracle's separated columns of the 16 (computed with the same criterion)
# and the median relative change of its x against the prior-free solve (the
# priors must move x well past the 1e-4 bar for the comparison to see them)
SEPARATED = {(0.01, 0.0): 16, (0.0, 2.0): 16, (0.01, 0.5): 16}
MEDIAN_CHANGE = {(0.01, 0.0): 3.36e-3, (0.0, 2.0): 2.29e-2, (0.01, 0.5): 8.52e-3}


@pytest.mark.parametrize("wt,wl", sorted(SEPARATED))
def test_image_priors_against_oracle(wt, wl):
    """A 64 x 16 image (power-law DCT columns, k = 6, m = 26, one Gaussian A)
    with the horizontal and vertical total variation, the local variation, or
    both."""
    b = W.image_batch(0.1, n=64, a=16, k=6)
    A = b.A
    Y = b.Y.T.astype(np.float64)
    print(f"image priors: w_tv {wt} w_lv {wl}", flush=True)
    sol, out = _solve(b, wt, wl)
    assert (out.status.cpu().numpy() == 0).all()
    base = clomp_image_fp64(A, Y, b.k, PARAMS, w_tv=f32(wt), w_lv=f32(wl))
    sep = _separated(A, Y, b.k, wt, wl, base)
    worst = 0.0
    for c in range(16):
        supp = out.support[c][: int(out.n_selected[c])].cpu().tolist()
        x = out.x[c].cpu().numpy().astype(np.float64)
        rn = float(out.resid_norm[c])
        assert abs(rn - fp64_resid(A, Y[:, c], supp, x)) <= 1e-9 * (1 + np.linalg.norm(Y[:, c]))
        if sep[c]:
            assert supp == base[c].support, (c, supp, base[c].support)
            e = rel_err(x, base[c].x)
            worst = max(worst, e)
            assert e <= 1e-4, (c, e)
    print(f"separated {sum(sep)}/16, worst rel.err {worst:.2e}")
    assert sum(sep) == SEPARATED[(wt, wl)]
    free = clomp_image_fp64(A, Y, b.k, PARAMS)
    change = np.median([rel_err(base[c].x, free[c].x) for c in range(16)])
    assert change >= 0.9 * MEDIAN_CHANGE[(wt, wl)], change
    sol.close()


def test_image_mode_without_priors_is_the_shared_schedule():
    """Weights 0: the columns decouple, and image mode (one Adam launch per
    step) gives the shared-dictionary schedule's supports and learned
    coefficients (CLOMP_FLAG_NO_REFINE; its Adam runs in support-sized
    workgroups, so only rounding differs)."""
    b = W.image_batch(0.1, n=64, a=16, k=6)
    s1, img = _solve(b, 0.0, 0.0)
    s2, ref = _solve(b, 0.0, 0.0, flags=C.FLAG_NO_REFINE | C.FLAG_NO_FUSED_SMALL)
    for c in range(16):
        assert img.support[c].tolist() == ref.support[c].tolist()
        assert rel_err(img.x[c].cpu().numpy().astype(np.float64),
                       ref.x[c].cpu().numpy().astype(np.float64)) <= 1e-5
    s1.close()
    s2.close()


def test_image_edges():
    """Two columns (no 3 x 3 window: the local variation vanishes) against the
    oracle; a zero column (empty support, x = 0) among live ones; batches the
    image mode refuses."""
    b = W.image_batch(0.1, n=64, a=2, k=6)
    A = b.A
    Y = b.Y.T.astype(np.float64)
    sol, out = _solve(b, 0.01, 1.0)
    base = clomp_image_fp64(A, Y, b.k, PARAMS, w_tv=f32(0.01), w_lv=f32(1.0))
    for c in range(2):
        assert out.support[c].tolist()[: b.k] == base[c].support
        assert rel_err(out.x[c].cpu().numpy().astype(np.float64), base[c].x) <= 1e-4
    sol.close()
    b = W.image_batch(0.1, n=64, a=8, k=6)
    Yz = b.Y.copy()
    Yz[3] = 0.0
    sol, out = _solve(b, 0.01, 0.5, Y=Yz)
    st = out.status.cpu().numpy()
    assert st[3] & C.ST_ZERO_Y and int(out.n_selected[3]) == 0 and not out.x[3].any()
    base = clomp_image_fp64(b.A, Yz.T.astype(np.float64), b.k, PARAMS, w_tv=f32(0.01),
                            w_lv=f32(0.5))
    assert base[3].support == []
    for c in (0, 1, 2, 4, 5, 6, 7):      # every oracle gap above 3e-3
        assert out.support[c].tolist()[: b.k] == base[c].support
        assert rel_err(out.x[c].cpu().numpy().astype(np.float64), base[c].x) <= 1e-4
    sol.close()
    # refused: different k per column, different A per column, OMP
    At = dev(b.At)
    items = [dict(At=At, m=b.m, y=dev(b.Y[c]), k=b.k + (c == 2)) for c in range(4)]
    sol = C.Solver(0, method="clomp", flags=C.FLAG_IMAGE, prior_tv=0.01)
    with pytest.raises(C.ClompError, match="NOT_SUPPORTED"):
        sol.solve_batch(items)
    items = [dict(At=dev(b.At), m=b.m, y=dev(b.Y[c]), k=b.k) for c in range(4)]
    with pytest.raises(C.ClompError, match="NOT_SUPPORTED"):
        sol.solve_batch(items)
    sol.close()
    with pytest.raises(C.ClompError, match="NOT_SUPPORTED"):
        C.Solver(0, method="omp", flags=C.FLAG_IMAGE)
    with pytest.raises(C.ClompError, match="NOT_SUPPORTED"):
        C.Solver(0, method="clomp", prior_lv=1.0)
