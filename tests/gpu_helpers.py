"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same stored inputs, and compare."""

import numpy as np
import torch

from oracle import ClompParams, clomp_fp64, omp_fp64, well_separated

f32 = lambda v: float(np.float32(v))

# The library takes float32 hyper-parameters; the oracle gets exactly those
# values so both sides use identical constants.
PARAMS = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9),
                     beta2=f32(0.999), eps_rel=f32(1e-8))

FP32_DELTA, FP32_U = 1e-4, 2.0 ** -24
BF16_DELTA, BF16_U = 1e-2, 2.0 ** -8


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_bf16(At32_t):
    return At32_t.to(torch.bfloat16)


def oracle_run(method, A, y, k, A_refine=None, params=PARAMS):
    if method == "omp":
        return omp_fp64(A, y, k)
    return clomp_fp64(A, y, k, params, A_refine=A_refine)


def oracle_final_x(method, A, y, k, A_refine=None, params=PARAMS):
    """The oracle's final x: OMP's least squares uses the same matrix as its
    selection; the GPU OMP refines on the master too, so compare against the
    master least squares on the oracle's support."""
    from oracle import lstsq_support
    res = oracle_run(method, A, y, k, A_refine, params)
    if A_refine is not None:
        x = np.zeros(A.shape[1])
        x[res.support] = lstsq_support(A_refine, y, res.support)
        res.x = x
    return res


def rel_err(x, ref):
    nr = np.linalg.norm(ref)
    return np.linalg.norm(x - ref) / (nr if nr > 0 else 1.0)


def coef_err(x, ref, floor=1e-2):
    """Per-coefficient companion of rel_err: the largest relative error over
    the significant coefficients of ref (|ref_j| >= floor * max |ref|), and
    the largest absolute error of any coefficient relative to ||ref||_2.  A
    normwise gate alone lets a small coefficient be wrong by 100%."""
    ref = np.asarray(ref, np.float64)
    x = np.asarray(x, np.float64)
    top = np.abs(ref).max() if ref.size else 0.0
    if top == 0.0:
        return 0.0, float(np.abs(x).max() if x.size else 0.0)
    sig = np.abs(ref) >= floor * top
    rel = float(np.max(np.abs(x[sig] - ref[sig]) / np.abs(ref[sig])))
    absn = float(np.max(np.abs(x - ref)) / np.linalg.norm(ref))
    return rel, absn


def fp64_resid(A, y, supp, x):
    S = list(supp)
    return float(np.linalg.norm(np.asarray(y, np.float64) - A[:, S] @ np.asarray(x, np.float64)[S]))


def compare(gpu, i, res, A_ref, y, *, delta, u, method, A_sel, k, tol_x, sep_params=PARAMS):
    """Compare instance i of a GPU BatchResult with an oracle result.
    Returns 'identical' (well separated, asserted), or 'skipped'."""
    supp_gpu = gpu.support[i][: int(gpu.n_selected[i])].cpu().numpy().tolist()
    x_gpu = gpu.x[i].cpu().numpy().astype(np.float64)
    # a7 closed form: the FP64 norm the library reports for its own x
    rn = float(gpu.resid_norm[i])
    assert abs(rn - fp64_resid(A_ref, y, supp_gpu, x_gpu)) <= 1e-9 * (1 + np.linalg.norm(y)), i
    ok, _ = well_separated(A_sel, y, k, method=method, params=sep_params, delta=delta, u=u,
                           A_refine=None if A_sel is A_ref else A_ref, base=res)
    if not ok:
        return "skipped"
    assert supp_gpu == res.support, (i, supp_gpu, res.support)
    e = rel_err(x_gpu, res.x)
    assert e <= tol_x, (i, e)
    # per coefficient: no coefficient of at least 1% of the largest is off by
    # more than 100 times the normwise tolerance
    ce, _ = coef_err(x_gpu, res.x)
    assert ce <= 100 * tol_x, (i, ce)
    return "identical"
