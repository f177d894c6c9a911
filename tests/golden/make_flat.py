"""Write flat_oracle.json: the FP64 oracle's results on the flattened 256 x 256
image as one signal (n = 65536, m = 19661, k = 2048, A iid N(0, 1/m) drawn on
the host by workloads.flat_image_host, power-law coefficients, noiseless).

  clomp  O2 on the stored bfloat16 values with the least-squares refinement on
         the float32 master (clomp_gram_fp64: the Gram-form rendering of O2;
         the plain one would take days here)
  omp    O1 on the float32 master (omp_cgs2_fp64: updated QR)
Separation, reported as the separated prefix of the ordered support (two
perturbation seeds per gate): the float32 gates (gap 1e-4, perturbation 2^-24)
for both methods, since each oracle sees the stored values and the library
differs from it only by float32 arithmetic; for CLOMP also the bfloat16 gates
(gap 1e-2, perturbation 2^-8).  Needs about 32 GB of memory and about
40 minutes on 8 cores.  Calls only the oracle and the seeded input generators:
    python tests/golden/make_flat.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import (ClompParams, clomp_gram_fp64, common_prefix, omp_cgs2_fp64,  # noqa: E402
                    perturbed_atoms, perturbed_vector, separated_prefix)
from paper_2501_11592_amd import workloads as W  # noqa: E402

f32 = lambda v: float(np.float32(v))
PARAMS = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                     eps_rel=f32(1e-8))


def log(msg):
    print(f"{time.strftime('%H:%M:%S')} {msg}", flush=True)


def main():
    m, k = W.FLAT_M, W.FLAT_K
    At, y, supp, s = W.flat_image_host()
    n = At.shape[0]
    out = {"workload": "flattened 256x256 image: n=65536, m=19661, k=2048 power-law, noiseless",
           "n": n, "m": m, "k": k, "A_sha256": W.fingerprint(At), "y_sha256": W.fingerprint(y),
           "params": {"inner_steps": 32, "lr_rel": 0.05, "beta1": 0.9, "beta2": 0.999,
                      "eps_rel": 1e-8}}
    log("inputs drawn")
    # atom-major float64 copies: the master values and the stored bfloat16 values
    Am = np.empty((n, m))
    Ab = np.empty((n, m))
    for j0 in range(0, n, W.FLAT_CHUNK):
        j1 = min(n, j0 + W.FLAT_CHUNK)
        Am[j0:j1] = At[j0:j1, :m]
        Ab[j0:j1] = W.bf16_values(At[j0:j1, :m])
    del At
    yv = y.astype(np.float64)
    P = np.empty((n, m))
    truth = set(supp.tolist())
    gates = {"fp32": (1e-4, 2.0 ** -24), "bf16": (1e-2, 2.0 ** -8)}
    for method, A, gnames in (("clomp", Ab, ("fp32", "bf16")), ("omp", Am, ("fp32",))):
        def run(AA, yy, refine):
            if method == "clomp":
                return clomp_gram_fp64(AA.T, yy, k, PARAMS, A_refine=refine)
            return omp_cgs2_fp64(AA.T, yy, k, A_refine=refine)
        t0 = time.time()
        base = run(A, yv, Am.T if method == "clomp" else None)
        dt = time.time() - t0
        log(f"{method}: base run {dt:.0f} s")
        rec = {"support": [int(j) for j in base.support],
               "x_support": [float(base.x[j]) for j in base.support],
               "resid_norm": base.resid_norm, "gaps": [float(g) for g in base.gaps],
               "oracle_seconds": dt, "truth_overlap": len(set(base.support) & truth) / k}
        for gname in gnames:
            delta, u = gates[gname]
            pert = []
            for sd in (1, 2):
                perturbed_atoms(A, u, sd, out=P)
                pert.append(run(P, perturbed_vector(yv, u, sd), None))
                log(f"{method}: {gname} perturbed run {sd}")
            rec[f"separated_prefix_{gname}"] = int(separated_prefix(base, pert, delta))
            rec[f"perturbed_common_prefix_{gname}"] = [common_prefix(base.support, p.support)
                                                       for p in pert]
        if method == "clomp":
            rec["s_adam"] = [float(v) for v in base.extra["s_adam"]]
        out[method] = rec
        with open(os.path.join(HERE, "flat_oracle.json"), "w") as f:
            json.dump(out, f)
        log(f"{method}: separated prefix {rec['separated_prefix_fp32']}, truth overlap "
            f"{rec['truth_overlap']:.3f}, resid {rec['resid_norm']:.3e}")


if __name__ == "__main__":
    main()
