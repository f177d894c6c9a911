"""Write uneven_oracle.json: the FP64 oracle's results on the stratified sample
of the uneven batch (4096 signals, n log-uniform in [512, 8192], m/n uniform in
[0.1, 0.5], k uniform in [n/64, n/16]; BF16 bulk with an FP32 master).  The
sixteen sampled signals are the ones the batch draws on the host
(workloads.uneven_golden_indices / uneven_instance_golden), so the GPU tests
and the benchmark solve exactly these inputs inside the full batch.

Per signal and method the oracle runs on the stored bfloat16 values (selection
and coefficient learning) and refines on the float32 master (least squares on
the support), as the library does:
  clomp  O2 clomp_fp64 (plain rendering), A_refine = master
  omp    O1 omp_fp64 on the bfloat16 values, least squares on the master
The oracle sees the stored bfloat16 values, so between it and the library only
the arithmetic differs (float32 accumulation of exact bfloat16 products on the
GPU): separation is recorded under the float32 gates (gap 1e-4, relative
perturbation 2^-24), which decide support identity for that path, and under the
bfloat16 gates (gap 1e-2, perturbation 2^-8) for paths that round operands to
bfloat16; two perturbation seeds each.  Calls only the oracle and the seeded
input generators:
    python tests/golden/make_uneven.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import (ClompParams, clomp_fp64, omp_fp64, lstsq_support,  # noqa: E402
                    resid_norm_fp64, separation_report)
from paper_2501_11592_amd import workloads as W  # noqa: E402

f32 = lambda v: float(np.float32(v))
PARAMS = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                     eps_rel=f32(1e-8))
GATES = {"fp32": (1e-4, 2.0 ** -24), "bf16": (1e-2, 2.0 ** -8)}


def separation(Ab, y, k, method, ref, Am=None):
    out = {}
    for name, (delta, u) in GATES.items():
        ok, pre, _ = separation_report(Ab, y, k, method=method, params=PARAMS, delta=delta, u=u,
                                       A_refine=Am, base=ref)
        out[f"separated_{name}"] = bool(ok)
        out[f"separated_prefix_{name}"] = int(pre)
    return out


def one(i, sp):
    sig = W.uneven_instance_golden(i, sp)
    m = sp.m
    Am = sig.At[:, :m].astype(np.float64).T                 # master values (m, n)
    Ab = W.bf16_values(sig.At[:, :m]).astype(np.float64).T  # stored bfloat16 values
    y = sig.y.astype(np.float64)
    rec = {"index": i, "n": sp.n, "m": m, "k": sp.k,
           "A_sha256": W.fingerprint(sig.At), "y_sha256": W.fingerprint(sig.y)}
    t0 = time.time()
    ref = clomp_fp64(Ab, y, sp.k, PARAMS, A_refine=Am)
    rec["clomp"] = {"support": [int(j) for j in ref.support],
                    "x_support": [float(ref.x[j]) for j in ref.support],
                    "s_adam": [float(v) for v in ref.extra["s_adam"]],
                    "resid_norm": ref.resid_norm, "min_gap": float(min(ref.gaps)),
                    "truth_overlap": len(set(ref.support) & set(sig.support.tolist())) / sp.k,
                    **separation(Ab, y, sp.k, "clomp", ref, Am)}
    oref = omp_fp64(Ab, y, sp.k)
    xo = lstsq_support(Am, y, oref.support)
    rec["omp"] = {"support": [int(j) for j in oref.support],
                  "x_support": [float(v) for v in xo],
                  "resid_norm": resid_norm_fp64(Am, y, oref.support, xo),
                  "min_gap": float(min(oref.gaps)),
                  "truth_overlap": len(set(oref.support) & set(sig.support.tolist())) / sp.k,
                  **separation(Ab, y, sp.k, "omp", oref)}
    rec["oracle_seconds"] = time.time() - t0
    return rec


def main():
    specs = W.uneven_specs(4096)
    idx = W.uneven_golden_indices(specs)
    out = {"workload": "uneven batch, stratified sample of 16 signals (bfloat16 bulk, float32 "
                       "master)",
           "params": {"inner_steps": 32, "lr_rel": 0.05, "beta1": 0.9, "beta2": 0.999,
                      "eps_rel": 1e-8},
           "separation": {name: {"delta": d, "u": u, "seeds": [1, 2]}
                          for name, (d, u) in GATES.items()},
           "instances": []}
    for i in idx:
        rec = one(i, specs[i])
        out["instances"].append(rec)
        c, o = rec["clomp"], rec["omp"]
        print(f"{i}: n={rec['n']} m={rec['m']} k={rec['k']} clomp prefix fp32/bf16 "
              f"{c['separated_prefix_fp32']}/{c['separated_prefix_bf16']} omp "
              f"{o['separated_prefix_fp32']}/{o['separated_prefix_bf16']} "
              f"{rec['oracle_seconds']:.1f}s", flush=True)
        with open(os.path.join(HERE, "uneven_oracle.json"), "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    main()
