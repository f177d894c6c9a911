"""Write large1d_oracle.json: the FP64 oracle's results on the large 1-D
workload (n=16384, m=4096, k=256, float32 A, seed 0), used as the expected
values of the full-size parity test and the benchmark's accuracy gate.

Calls only the oracle and the seeded input generator:
    python tests/golden/make_large1d.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ClompParams, clomp_fp64, omp_fp64, well_separated  # noqa: E402
from paper_2501_11592_amd import workloads as W  # noqa: E402

f32 = lambda v: float(np.float32(v))
PARAMS = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                     eps_rel=f32(1e-8))


def main():
    sig = W.single_large(0)
    A = sig.A
    out = {"workload": "large1d", "n": sig.n, "m": sig.m, "k": sig.k, "seed": 0,
           "params": {"inner_steps": 32, "lr_rel": 0.05, "beta1": 0.9, "beta2": 0.999,
                      "eps_rel": 1e-8}}
    for method in ("clomp", "omp"):
        t0 = time.time()
        res = clomp_fp64(A, sig.y, sig.k, PARAMS) if method == "clomp" else omp_fp64(A, sig.y, sig.k)
        dt = time.time() - t0
        ok, _ = well_separated(A, sig.y, sig.k, method=method, params=PARAMS, delta=1e-4,
                               u=2.0 ** -24, base=res)
        out[method] = {"support": [int(j) for j in res.support],
                       "x_support": [float(res.x[j]) for j in res.support],
                       "resid_norm": res.resid_norm, "min_gap": float(min(res.gaps)),
                       "well_separated": bool(ok), "oracle_seconds": dt,
                       "truth_rel_err": float(np.linalg.norm(res.x - sig.s) / np.linalg.norm(sig.s))}
        print(method, "done", dt, "s; well separated:", ok, flush=True)
    with open(os.path.join(HERE, "large1d_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
