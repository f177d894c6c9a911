"""The allocation-free gradient entry point (clomp_grad_noalloc) against
clomp_grad on the same inputs: two calls in a row, the second smaller, so the
second runs on scratch the first left behind.  Both entry points run the same
kernels with the same column chunks, so the results agree bit for bit; the FP64
oracle gradient pins both."""

import numpy as np
import pytest
import torch

from oracle import grad_fp64
from paper_2501_11592_amd import clomp as C
from paper_2501_11592_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(n, m, seed, dtype):
    g = np.random.default_rng([2501, 11592, 77, seed])
    lda = W.pad_lda(m, 8 if dtype == torch.float64 else 4)
    At = np.zeros((n, lda))
    At[:, :m] = g.standard_normal((n, m)) / np.sqrt(m)
    x = g.standard_normal(n)
    mask = (g.random(n) < 0.3).astype(np.uint8)
    y = g.standard_normal(m)
    dev = lambda a, dt=dtype: torch.as_tensor(a, dtype=dt, device="cuda")
    return (At, x, mask, y), (dev(At), dev(x), dev(mask, torch.uint8), dev(y))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_grad_matches_grad_twice(dtype):
    sol = C.Solver(0)
    go = torch.tensor(0.75, dtype=dtype, device="cuda")
    # 3000 atoms: 12 column chunks with a ragged tail; m = 700 spans 11 row tiles
    for n, m, seed in ((3000, 700, 1), (517, 93, 2)):
        host, (At, x, mask, y) = _case(n, m, seed, dtype)
        print(f"noalloc grad: dtype {dtype} n={n} m={m} seed {seed}", flush=True)
        ref = sol.grad(At, m, x, mask, y, grad_out=go)
        got = sol.grad(At, m, x, mask, y, grad_out=go, noalloc=True)
        # the same call without a residual output keeps it in the scratch
        got_nu = sol.grad(At, m, x, mask, y, grad_out=go, want_resid=False, noalloc=True)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert torch.equal(ref[0], got_nu[0]) and torch.equal(ref[1], got_nu[1])
        A64 = host[0][:, :m].T
        l64, g64, u64 = grad_fp64(host[1], host[2], A64, host[3])
        tol = 1e-12 if dtype == torch.float64 else 1e-5
        gn = got[1].double().cpu().numpy()
        scale = np.linalg.norm(g64) * 0.75
        assert np.linalg.norm(gn - 0.75 * g64) <= tol * scale
        assert abs(got[0].item() - l64) <= tol * l64
    sol.close()


def test_noalloc_grad_rejects_beyond_its_scratch():
    sol = C.Solver(0)
    n, m = 65536, 16384          # 256 chunks x 16384 rows x 4 B > 16 MiB
    At = torch.empty((n, m), dtype=torch.float32, device="cuda")
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    mask = torch.zeros(n, dtype=torch.uint8, device="cuda")
    y = torch.zeros(m, dtype=torch.float32, device="cuda")
    with pytest.raises(C.ClompError, match="INVALID_ARGUMENT.*scratch"):
        sol.grad(At, m, x, mask, y, noalloc=True)
    # m = 16320 is the largest that fits at n = 65536 (the header's example);
    # with an empty mask no atom is read, so the uninitialised A is harmless
    loss, gx, u = sol.grad(At, 16320, x, mask, y, noalloc=True)
    torch.cuda.synchronize()
    assert loss.item() == 0.0 and not gx.any() and not u.any()
    del At
    sol.close()
