"""Benchmark: CLOMP signals/s on one MI355X next to plain GPU OMP on the same
instances, with the roofline of the dominant kernel and the FP64 CPU oracle
timed on the host.

Default workload (the largest that fits one GPU): the uneven batch, 4096
signals with n log-uniform in [512, 8192], m/n uniform in [0.1, 0.5], k
uniform in [n/64, n/16], A iid N(0, 1/m) stored as a BF16 bulk copy (greedy
loop) and an FP32 master (refinement and FP64 residual norm), N(0, 1)
non-zeros, noiseless; all 4096 in one call.  Accuracy is stated against the
FP64 oracle's stored results on the batch's sixteen stratified signals
(tests/golden/uneven_oracle.json).

Other workloads (--workload): large1d (one signal n=16384, m=4096, k=256,
float32: every iteration streams the whole 268 MB dictionary), small1d (1000
signals n=256 m=64 k=8), image (256 columns sharing A, sampling rate
0.1/0.3/0.5), image4k (3840 columns of n=2160 sharing A, k=108: the
shared-dictionary schedule), flat (n=65536, m=19661, k=2048, BF16 CLOMP vs
FP32 OMP).

A step is one full solve of the workload's batch (k greedy iterations,
refinement, FP64 residual norm) through the C ABI, inputs resident in HBM.
W untimed warm-up steps, then K timed steps between device synchronisations.
Prints one JSON line.

    python bench.py [--workload uneven] [--steps K] [--warmup W] [--gpus 1]
                    [--no-cpu-baseline] [--no-graph]
"""

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "signals/sec CLOMP vs plain OMP on GPU at rel.err≤1e-3; HBM GB/s / MFMA util"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 5 for the uneven and flat workloads, else 30)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default: 1 for the uneven and flat workloads, else 3)")
    ap.add_argument("--workload", default="uneven",
                    choices=["large1d", "small1d", "image", "image4k", "uneven", "flat"])
    ap.add_argument("--sr", type=float, default=0.3, help="image workload sampling rate")
    ap.add_argument("--bf16", action="store_true",
                    help="image4k: BF16 bulk copy of A with the float32 values as master")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-iht", action="store_true", help="skip the IHT comparison leg")
    ap.add_argument("--iht", action="store_true",
                    help="uneven workload: also run the IHT leg (off by default there)")
    ap.add_argument("--paper", action="store_true",
                    help="uneven workload: also run the paper-mode leg (off by default there)")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper-mode CLOMP leg (T_h = 0.7, 200 iterations)")
    ap.add_argument("--flow", default="auto", choices=["auto", "resid", "corr"],
                    help="schedule: library default, residual, or correlation update")
    ap.add_argument("--no-shared-gram", action="store_true",
                    help="keep per-signal passes over a shared A (no full Gram matrix)")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--pass-tile-kb", type=int, default=0,
                    help="bulk-matrix KB per pass workgroup (0: the library default)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its tile candidates on the first call")
    ap.add_argument("--image-priors", type=float, nargs=2, default=None, metavar=("W_TV", "W_LV"),
                    help="image workload: also run CLOMP on the columns as one image with "
                         "the 2-D total variation and local variation weights given")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 1 GiB (reference for HBM counters)")
    args = ap.parse_args()
    big = args.workload in ("uneven", "flat")
    if args.steps is None:
        args.steps = 5 if big else 30
    if args.warmup is None:
        args.warmup = 1 if big else 3
    return args


def copy_calibration(torch):
    """Five plain device-to-device copies of 1 GiB: 1 GiB read and 1 GiB
    written per copy kernel, the reference for scaling FETCH_SIZE/WRITE_SIZE."""
    n = (1 << 30) // 4
    src = torch.randn(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "ms_per_copy": 1e3 * dt, "GBps_read_plus_write": 8 * n / dt / 1e9}))


def f32(v):
    return float(np.float32(v))


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ workloads
def build_workload(args, torch, W):
    """Returns dict(name, desc, cfg, clomp_items, omp_items, dtype, host)."""
    dev = torch.device("cuda", 0)
    if args.workload == "large1d":
        sig = W.single_large(0)
        it = dict(At=torch.from_numpy(sig.At).to(dev), m=sig.m,
                  y=torch.from_numpy(sig.y).to(dev), k=sig.k)
        return dict(name="large1d",
                    desc="large 1-D signal: n=16384, m=4096, k=256, A iid N(0,1/m) float32, "
                         "noise N(0,1e-4), batch 1",
                    cfg=dict(n=sig.n, m=sig.m, k=sig.k, batch=1),
                    clomp_items=[it], omp_items=[it], dtype="f32", host=[sig])
    if args.workload == "small1d":
        sigs = [W.single_small(i) for i in range(1000)]
        items = [dict(At=torch.from_numpy(s.At).to(dev), m=s.m, y=torch.from_numpy(s.y).to(dev),
                      k=s.k) for s in sigs]
        return dict(name="small1d",
                    desc="1000 single 1-D signals n=256, m=64, k=8, A iid N(0,1/m), noiseless, "
                         "one batch",
                    cfg=dict(n=256, m=64, k=8, batch=1000), clomp_items=items, omp_items=items,
                    dtype="f32", host=sigs)
    if args.workload == "image":
        b = W.image_batch(args.sr)
        At = torch.from_numpy(b.At).to(dev)
        Y = torch.from_numpy(b.Y).to(dev)
        items = [dict(At=At, m=b.m, y=Y[c], k=b.k) for c in range(Y.shape[0])]
        return dict(name=f"image_sr{args.sr}",
                    desc=f"256 columns of a synthetic 256x256 image sharing one Gaussian A, "
                         f"sampling rate {args.sr} (m={b.m}), power-law k=32, float32",
                    cfg=dict(n=b.n, m=b.m, k=b.k, batch=256, shared_A=True),
                    clomp_items=items, omp_items=items, dtype="f32", host=b)
    if args.workload == "image4k":
        log("drawing the 4K-scale image batch (3840 columns, n=2160)")
        b = W.image4k_batch(args.sr)
        At = torch.from_numpy(b.At).to(dev)
        Y = torch.from_numpy(b.Y).to(dev)
        if args.bf16:
            # BF16 bulk copy (the contractions on the BF16 matrix cores) with the
            # float32 values as the master of the refinement
            Ab = torch.zeros((b.n, W.pad_lda(b.m, 2)), dtype=torch.bfloat16, device=dev)
            Ab[:, :b.m] = At[:, :b.m].to(torch.bfloat16)
            items = [dict(At=Ab, At_master=At, m=b.m, y=Y[c], k=b.k) for c in range(Y.shape[0])]
        else:
            items = [dict(At=At, m=b.m, y=Y[c], k=b.k) for c in range(Y.shape[0])]
        dt = "bf16" if args.bf16 else "f32"
        return dict(name=f"image4k_sr{args.sr}",
                    desc=f"3840 columns of a synthetic 3840x2160 image sharing one Gaussian A, "
                         f"sampling rate {args.sr} (m={b.m}), power-law k={b.k}, "
                         + ("BF16 bulk + FP32 master" if args.bf16 else "float32"),
                    cfg=dict(n=b.n, m=b.m, k=b.k, batch=3840, shared_A=True),
                    clomp_items=items, omp_items=items, dtype=dt, host=b)
    if args.workload == "uneven":
        log("drawing the uneven batch on the device (4096 signals, ~89 GB)")
        specs, items, supps, coefs = W.uneven_batch_device(4096, dev)
        tot = sum(sp.n * sp.m for sp in specs)
        return dict(name="uneven",
                    desc="4096 signals, n log-uniform [512,8192], m/n U[0.1,0.5], k U[n/64,n/16], "
                         "A iid N(0,1/m): BF16 bulk + FP32 master",
                    cfg=dict(batch=4096, sum_mn=tot), clomp_items=items, omp_items=items,
                    dtype="bf16", host=(specs, supps, coefs))
    if args.workload == "flat":
        log("drawing the flattened-image matrix on the device (5.2 GB FP32 + 2.6 GB BF16)")
        Am, Ab, y, supp, s = W.flat_image_device(dev)
        c_it = dict(At=Ab, m=W.FLAT_M, y=y, k=W.FLAT_K, At_master=Am)
        o_it = dict(At=Am, m=W.FLAT_M, y=y, k=W.FLAT_K)
        return dict(name="flat",
                    desc="flattened 256x256 image as one signal: n=65536, m=19661, k=2048 "
                         "power-law; BF16 CLOMP (FP32 refinement) vs FP32 OMP",
                    cfg=dict(n=W.FLAT_N, m=W.FLAT_M, k=W.FLAT_K, batch=1),
                    clomp_items=[c_it], omp_items=[o_it], dtype="bf16", host=(supp, s))
    raise SystemExit(f"unknown workload {args.workload}")


def kernel_digest():
    """Digest of the device code behind the dominant kernels (coefficient
    bodies, the pass and scan kernels of the correlation-update schedule and
    the shared device header)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2501_11592_amd", "csrc", "solve_kernels.hip")).read()
    hdr = open(os.path.join(ROOT, "paper_2501_11592_amd", "csrc", "dev_common.h")).read()
    mark = "// ============================================================ "
    def region(a, b):
        return src[src.index(mark + a):src.index(mark + b)]
    text = region("Adam (CLOMP)", "rows kernels") + \
        region("correlation-update schedule", "image priors") + hdr
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel's device code has changed since it was measured."""
    f = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(f) or not kernel.startswith("coef_pass"):
        return None
    d = json.load(open(f))
    return d["traffic_bytes_per_launch"] if d.get("kernel_digest") == kernel_digest() else None


VALU_PEAK_TFLOPS = 157.3   # FP32 vector, 256 CUs at 2.4 GHz
MFMA_FP32_PEAK_TFLOPS = 157.3   # dense FP32 matrix cores (published)
MFMA_BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix cores (published, without sparsity)


def fused_flops(items, method, inner_steps=32):
    """Algorithmic FP32 operations of the fused small-signal loop over a batch:
    per iteration t the scan (2mn), the new Gram column and b (2m(t+2)), the
    coefficient update (T steps of 2(t+1)^2 + 10(t+1) for Adam; 6t^2 for the
    bordered inverse) and the residual (2m(t+1))."""
    tot = 0.0
    for it in items:
        n, m, k = int(it["At"].shape[0]), int(it["m"]), int(it["k"])
        ke = min(k, m, n)
        for t in range(ke):
            tot += 2.0 * m * n + 2.0 * m * (t + 2) + 2.0 * m * (t + 1)
            if method == "clomp":
                tot += inner_steps * (2.0 * (t + 1) ** 2 + 10.0 * (t + 1))
            else:
                tot += 6.0 * t * t
    return tot


def roofline(p, items=None, method="clomp"):
    """Dominant launch of a profile (most total device time) and its achieved
    algorithmic bandwidth (or, for the fused small-signal loop, which works
    from LDS, its achieved FP32 rate)."""
    if p["launches"].get("fused", 0) > 0 and p["ms"]["fused"] >= max(p["ms"]["pass"],
                                                                      p["ms"]["scan"]):
        nl, ms = p["launches"]["fused"], p["ms"]["fused"]
        fl = fused_flops(items, method)   # one fused launch per solve
        k_ms = ms / nl
        ach = fl / (k_ms * 1e-3) / 1e12
        return {"kernel": "small_loop_kernel (whole greedy loop per signal, dictionary in LDS)",
                "bound": "alu", "achieved": ach, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / VALU_PEAK_TFLOPS, "traffic": None, "avg_launch_us": 1e3 * k_ms,
                "flops_per_launch": fl, "hbm_bytes_per_launch": p["fused_bytes"] / nl,
                "launches": nl}
    shared = (items is not None and len(items) > 1 and p["pass_bytes"] == 0 and
              len({it["At"].data_ptr() for it in items}) == 1)
    if shared and p["ms"]["scan"] > max(p["ms"]["pass"], p["ms"]["coef"]):
        # shared dictionary: the scan is the contraction C = A^T R of the whole
        # batch on the FP32 matrix cores (plus the once-per-solve A^T A, A^T Y)
        n, m = int(items[0]["At"].shape[0]), int(items[0]["m"])
        nl, ms = p["launches"]["scan"], p["ms"]["scan"]
        fl = 2.0 * n * m * len(items)
        k_ms = ms / nl
        ach = fl / (k_ms * 1e-3) / 1e12
        what = ("C = A^T R over the batch, argmax epilogue" if method in ("clomp", "omp")
                else "gradient G = A^T R over the batch")
        # the scan of a BF16 bulk matrix runs on the BF16 matrix cores (the
        # IHT / paper-mode gradient stays on FP32)
        bfs = str(items[0]["At"].dtype) == "torch.bfloat16" and method in ("clomp", "omp")
        peak = MFMA_BF16_PEAK_TFLOPS if bfs else MFMA_FP32_PEAK_TFLOPS
        kname = "shared_mfma_bf16_kernel" if bfs else "shared_mfma_kernel"
        return {"kernel": f"{kname} ({what})",
                "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": None,
                "avg_launch_us": 1e3 * k_ms, "flops_per_launch": fl, "launches": nl}
    if shared and p["launches"]["coef"] > 0 and p["ms"]["coef"] >= p["ms"]["scan"]:
        # shared dictionary: the launches carry coefficient workgroups only
        nl, ms = p["launches"]["coef"], p["ms"]["coef"]
        fl = 0.0
        for it in items:
            ke = min(int(it["k"]), int(it["m"]), int(it["At"].shape[0]))
            for t in range(ke):
                fl += (32 * (2.0 * (t + 1) ** 2 + 10.0 * (t + 1)) if method == "clomp"
                       else 6.0 * t * t)
        k_ms = ms / nl
        ach = fl / nl / (k_ms * 1e-3) / 1e12
        return {"kernel": ("coef_reg_kernel" if method == "clomp" else "coef_omp_kernel")
                + " (support-sized coefficient workgroups: shared dictionary)",
                "bound": "alu", "achieved": ach, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / VALU_PEAK_TFLOPS, "traffic": None, "avg_launch_us": 1e3 * k_ms,
                "flops_per_launch": fl / nl, "launches": nl}
    if p["launches"]["pass"] > 0 and p["ms"]["pass"] >= p["ms"]["scan"]:
        name = "coef_pass_kernel (Adam/OMP block + pass h = A^T a_j over A)"
        nl, ms, byt = p["launches"]["pass"], p["ms"]["pass"], p["pass_bytes"]
    else:
        name = ("iht_grad_kernel (A^T r over A)" if method == "iht" else
                "cscan/ypass kernels (c = c0 - H s, argmax)" if p["launches"]["pass"] > 0
                else "scan_reg_kernel (c = A^T r, |c|, argmax)")
        nl, ms, byt = max(1, p["launches"]["scan"]), p["ms"]["scan"], p["scan_bytes"]
    k_ms = ms / nl
    bpl = byt / nl
    ach = bpl / (k_ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "avg_launch_us": 1e3 * k_ms,
            "bytes_per_launch": bpl, "launches": nl}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not served "
              "(independent signals shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2501_11592_amd import clomp as C
    from paper_2501_11592_amd import workloads as W

    log(f"workload {args.workload}")
    wl = build_workload(args, torch, W)
    torch.cuda.synchronize()
    # the uneven batch launches eagerly on the current stream (no graph
    # capture) and runs only the CLOMP and OMP legs unless --iht / --paper ask
    # for more; the other workloads replay captured graphs on a created stream
    uneven = wl["name"] == "uneven"
    if uneven:
        args.no_graph = True
        args.no_iht = not args.iht
        args.no_paper = not args.paper
    stream = (torch.cuda.current_stream(torch.device("cuda", 0)) if args.no_graph
              else torch.cuda.Stream(torch.device("cuda", 0)))
    flow_flag = {"auto": 0, "resid": C.FLAG_RESIDUAL_FLOW, "corr": C.FLAG_CORR_FLOW}[args.flow]
    flow_flag |= C.FLAG_NO_SHARED_GRAM if args.no_shared_gram else 0
    flow_flag |= C.FLAG_AUTOTUNE if args.autotune else 0
    flags = (0 if args.no_graph else C.FLAG_GRAPH) | flow_flag
    methods = ("clomp", "omp") + (() if args.no_iht else ("iht",)) + (
        () if args.no_paper else ("clomp_paper",))
    # the image leg: the columns coupled by the priors of Eq. (6) and (7)
    image_leg = args.image_priors is not None and wl["name"].startswith("image_sr")
    if args.image_priors is not None and not image_leg:
        raise SystemExit("--image-priors needs --workload image")
    methods += ("clomp_image",) if image_leg else ()

    def make_solver(m, fl):
        if m == "clomp_image":
            return C.Solver(0, method="clomp", flags=fl | C.FLAG_IMAGE,
                            prior_tv=args.image_priors[0], prior_lv=args.image_priors[1])
        return C.Solver(0, method=m, flags=fl)

    solvers = {m: make_solver(m, flags) for m in methods}
    if args.pass_tile_kb:
        for sv in solvers.values():
            sv.set_tuning(pass_tile_kb=args.pass_tile_kb)
    # IHT (200 iterations, the experiments' comparison method) runs on the
    # same storage as CLOMP
    items = {"clomp": wl["clomp_items"], "omp": wl["omp_items"], "iht": wl["clomp_items"],
             "clomp_paper": wl["clomp_items"], "clomp_image": wl["clomp_items"]}
    count = len(items["clomp"])

    # descriptors and outputs packed once (inputs stay resident); every step
    # launches the whole batch through the C ABI
    preps = {m: solvers[m].prepare(items[m], stream=stream) for m in methods}
    timings, outs = {}, {}
    for method in methods:
        log(f"{method} warmup {args.warmup}")
        for _ in range(args.warmup):
            solvers[method].run(preps[method], stream=stream)
        torch.cuda.synchronize()
        # no collector pause inside the timed region (a full collection over
        # the batch's descriptors takes tens of milliseconds)
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = solvers[method].run(preps[method], stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        gc.enable()
        timings[method] = dt / args.steps
        outs[method] = out
        log(f"{method} {1e3 * dt / args.steps:.3f} ms/step")

    # live per-phase timing with HIP events on the launch stream (no graph);
    # --profile-steps 0 skips it (runs under hardware-counter collection)
    prof = {}
    for method in (methods if args.profile_steps > 0 else ()):
        ps = make_solver(method, C.FLAG_PROFILE | flow_flag)
        if args.pass_tile_kb:
            ps.set_tuning(pass_tile_kb=args.pass_tile_kb)
        pp = ps.prepare(items[method], stream=stream)
        ps.run(pp, stream=stream)
        torch.cuda.synchronize()
        ps.profile_reset()
        for _ in range(args.profile_steps):
            ps.run(pp, stream=stream)
        torch.cuda.synchronize()
        prof[method] = ps.profile_read()
        ps.close()

    acc, cpu = {}, None
    if wl["name"] == "uneven":
        acc, cpu = accuracy_uneven(args, wl, outs)
    elif wl["name"] == "large1d":
        acc, cpu = accuracy_large1d(args, wl, outs)
    elif wl["name"] == "small1d" and not args.no_cpu_baseline:
        acc, cpu = accuracy_batch_sample(wl, outs, n_sample=200)
    elif wl["name"].startswith("image") and not args.no_cpu_baseline:
        acc, cpu = accuracy_shared_sample(wl, outs, *((24, 8) if wl["name"].startswith("image4k")
                                                      else (256, 256)))

    st = {m: outs[m].status.cpu().numpy() for m in outs}
    line = {
        "metric": METRIC,
        "value": count / timings["clomp"],
        "unit": "signals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * timings["clomp"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl["dtype"],
        "data": "synthetic",
        "config": dict(workload=wl["desc"], method="clomp", inner_steps=32,
                       graph=not args.no_graph, flow=args.flow, **wl["cfg"]),
        "omp": {"value": count / timings["omp"], "unit": "signals/s",
                "ms_per_step": 1e3 * timings["omp"],
                "dtype": "f32" if wl["name"] == "flat" else wl["dtype"]},
        "clomp_vs_omp": timings["omp"] / timings["clomp"],
        "iht": ({"value": count / timings["iht"], "unit": "signals/s",
                 "ms_per_step": 1e3 * timings["iht"], "iterations": 200,
                 "dtype": wl["dtype"]} if "iht" in timings else None),
        "clomp_paper": ({"value": count / timings["clomp_paper"], "unit": "signals/s",
                         "ms_per_step": 1e3 * timings["clomp_paper"], "iterations": 200,
                         "threshold": 0.7, "dtype": wl["dtype"]}
                        if "clomp_paper" in timings else None),
        "clomp_image": ({"value": count / timings["clomp_image"], "unit": "signals/s",
                         "ms_per_step": 1e3 * timings["clomp_image"],
                         "prior_tv": args.image_priors[0], "prior_lv": args.image_priors[1],
                         "dtype": wl["dtype"]} if "clomp_image" in timings else None),
        "accuracy": acc,
        "accuracy_gate_1e-3": (all(a["rel_err"] is not None and a["rel_err"] <= 1e-3
                                   for a in acc.values()) if acc else None),
        "status_flags_nonzero": {m: int((st[m] != 0).sum()) for m in st},
        "phase_ms_per_step": {m: {k: v / args.profile_steps for k, v in prof[m]["ms"].items()}
                              for m in prof},
        "roofline": roofline(prof["clomp"], items["clomp"], "clomp") if prof else None,
        "roofline_omp": roofline(prof["omp"], items["omp"], "omp") if prof else None,
        "roofline_iht": roofline(prof["iht"], items["iht"], "iht") if "iht" in prof else None,
        "roofline_clomp_paper": (roofline(prof["clomp_paper"], items["clomp_paper"], "iht")
                                 if "clomp_paper" in prof else None),
        "cpu_baseline": cpu,
    }
    if line["roofline"] is not None:
        line["roofline"]["traffic"] = measured_traffic(wl["name"], line["roofline"]["kernel"])
    print(json.dumps(line), flush=True)
    for s in solvers.values():
        s.close()


def _threads():
    from threadpoolctl import threadpool_info
    return int(max([p.get("num_threads", 1) for p in threadpool_info()] or [1]))


UNEVEN_CPU_STRATA = tuple(range(4, 15))   # golden-sample positions timed for the CPU baseline


def accuracy_uneven(args, wl, outs):
    """The batch's sixteen stratified signals (drawn on the host, one per
    sixteenth of the batch sorted by n) against the FP64 oracle's stored
    results, and the oracle timed on a bounded stratified sample of them as
    the CPU baseline (all host threads, then one)."""
    from paper_2501_11592_amd import workloads as W
    specs = wl["host"][0]
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "uneven_oracle.json")))
    acc = {}
    for method in ("clomp", "omp"):
        o = outs[method]
        rows = []
        for rec in gold["instances"]:
            i, g = rec["index"], rec[method]
            S = o.support[i][: int(o.n_selected[i])].cpu().tolist()
            xr = np.zeros(rec["n"])
            xr[g["support"]] = g["x_support"]
            x = o.x[i].cpu().numpy().astype(np.float64)
            rows.append((S == g["support"], bool(g["separated_fp32"]),
                         float(np.linalg.norm(x - xr) / np.linalg.norm(xr))))
        same = [e for ok, _, e in rows if ok]
        acc[method] = {
            "rel_err": float(max(same)) if same else None,
            "rel_err_median": float(np.median(same)) if same else None,
            "rel_err_all_max": float(max(e for _, _, e in rows)),
            "support_identical_fraction": len(same) / len(rows),
            "separated_fraction": sum(sep for _, sep, _ in rows) / len(rows),
            "sample": f"{len(rows)} stratified signals of the batch (one per sixteenth by n, "
                      "n = 564 .. 8189) against the stored FP64 oracle results; rel_err over "
                      "the signals whose ordered support equals the oracle's"}
    cpu = None if args.no_cpu_baseline else cpu_baseline_uneven(specs, gold, W)
    return acc, cpu


def cpu_baseline_uneven(specs, gold, W):
    """The FP64 CLOMP oracle (selection and Adam on the stored bfloat16
    values, least squares on the float32 master) timed on a stratified sample
    of the golden signals, with every host thread and with one, and scaled to
    the whole batch by sum(k m n) (an extrapolation: the sample's time times
    the batch's sum of k m n over the sample's)."""
    from oracle import clomp_fp64, ClompParams
    from threadpoolctl import threadpool_limits
    params = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                         eps_rel=f32(1e-8))
    recs = [gold["instances"][q] for q in UNEVEN_CPU_STRATA]
    cases = []
    for rec in recs:
        i = rec["index"]
        sig = W.uneven_instance_golden(i, specs[i])
        m = specs[i].m
        cases.append((W.bf16_values(sig.At[:, :m]).astype(np.float64).T,
                      sig.At[:, :m].astype(np.float64).T, sig.y.astype(np.float64), sig.k))

    def timed():
        t0 = time.perf_counter()
        for Ab, Am, y, k in cases:
            clomp_fp64(Ab, y, k, params, A_refine=Am)
        return time.perf_counter() - t0

    kmn = lambda sp: float(sp.k) * sp.m * sp.n
    scale = sum(kmn(sp) for sp in specs) / sum(kmn(specs[r["index"]]) for r in recs)
    log(f"timing the FP64 oracle on {len(cases)} stratified signals (all threads, then one)")
    threads = _threads()
    t_all = timed()
    with threadpool_limits(limits=1):
        t_one = timed()
    desc = ", ".join(f"n={specs[r['index']].n} m={specs[r['index']].m} k={specs[r['index']].k}"
                     for r in recs)
    return {"value": len(specs) / (t_all * scale), "unit": "signals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(cases)} stratified signals of the batch ({desc}) solved by the FP64 "
                      f"CLOMP oracle in {t_all:.1f} s, extrapolated to the 4096 signals by "
                      f"sum(k*m*n) (factor {scale:.0f})",
            "seconds": t_all, "host_cpus": os.cpu_count(),
            "one_core": {"value": len(specs) / (t_one * scale), "unit": "signals/s", "cores": 1,
                         "seconds": t_one}}


def accuracy_large1d(args, wl, outs):
    """rel.err against the FP64 oracle; the oracle solve is also the CPU
    baseline (one full solve of the benchmark signal, about 15 s)."""
    from oracle import clomp_fp64, ClompParams
    sig = wl["host"][0]
    golden = os.path.join(ROOT, "tests", "golden", "large1d_oracle.json")
    gold = json.load(open(golden)) if os.path.exists(golden) else None
    refs, cpu = {}, None
    if not args.no_cpu_baseline:
        params = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9),
                             beta2=f32(0.999), eps_rel=f32(1e-8))
        log("timing the FP64 oracle (one full CLOMP solve of this signal)")
        t0 = time.perf_counter()
        ref = clomp_fp64(sig.A, sig.y, sig.k, params)
        cdt = time.perf_counter() - t0
        cpu = {"value": 1.0 / cdt, "unit": "signals/s", "cores": _threads(), "kind": "oracle",
               "sample": "one full solve of the benchmark signal (n=16384, m=4096, k=256) by the "
                         "FP64 CLOMP oracle (NumPy/SciPy BLAS)",
               "seconds": cdt, "host_cpus": os.cpu_count()}
        refs["clomp"] = (ref.support, ref.x)
    if gold is not None:
        for method in ("clomp", "omp"):
            x = np.zeros(sig.n)
            x[gold[method]["support"]] = gold[method]["x_support"]
            refs.setdefault(method, (gold[method]["support"], x))
    acc = {}
    for method, (supp, xr) in refs.items():
        o = outs[method]
        xs = o.x[0].cpu().numpy().astype(np.float64)
        sg = o.support[0][: int(o.n_selected[0])].cpu().tolist()
        acc[method] = {"rel_err": float(np.linalg.norm(xs - xr) / np.linalg.norm(xr)),
                       "support_identical": sg == list(supp),
                       "support_set_equal": sorted(sg) == sorted(supp),
                       "truth_rel_err": float(np.linalg.norm(xs - sig.s) / np.linalg.norm(sig.s))}
    return acc, cpu


def accuracy_batch_sample(wl, outs, n_sample):
    """rel.err of a sample of a host-generated batch against the oracle, and
    the oracle's rate on that sample as the CPU baseline."""
    from oracle import clomp_fp64, omp_fp64, ClompParams
    params = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                         eps_rel=f32(1e-8))
    sigs = wl["host"][:n_sample]
    errs = {"clomp": [], "omp": []}
    same = {"clomp": 0, "omp": 0}
    t0 = time.perf_counter()
    refs = [clomp_fp64(s.A, s.y, s.k, params) for s in sigs]
    cdt = time.perf_counter() - t0
    orefs = [omp_fp64(s.A, s.y, s.k) for s in sigs]
    for method, rr in (("clomp", refs), ("omp", orefs)):
        o = outs[method]
        for i, r in enumerate(rr):
            xs = o.x[i].cpu().numpy().astype(np.float64)
            errs[method].append(np.linalg.norm(xs - r.x) / np.linalg.norm(r.x))
            same[method] += o.support[i][: int(o.n_selected[i])].cpu().tolist() == r.support
    acc = {m: {"rel_err": float(np.max(errs[m])), "rel_err_median": float(np.median(errs[m])),
               "support_identical_fraction": same[m] / len(sigs), "sample": len(sigs)}
           for m in errs}
    cpu = {"value": len(sigs) / cdt, "unit": "signals/s", "cores": _threads(), "kind": "oracle",
           "sample": f"{len(sigs)} of the 1000 signals, FP64 CLOMP oracle", "seconds": cdt,
           "host_cpus": os.cpu_count()}
    return acc, cpu


def accuracy_shared_sample(wl, outs, n_sample, n_omp):
    """Columns of a shared-dictionary image batch, evenly spaced, against the
    FP64 oracles (with a BF16 bulk copy: selection and Adam on the BF16 values,
    least squares on the float32 master); the CLOMP oracle's rate on them is
    the CPU baseline (all host threads, then one).  OMP is checked on the first
    n_omp of them (its oracle is the slower one)."""
    from oracle import clomp_fp64, omp_fp64, ClompParams
    from threadpoolctl import threadpool_limits
    from paper_2501_11592_amd import workloads as W
    params = ClompParams(inner_steps=32, lr_rel=f32(0.05), beta1=f32(0.9), beta2=f32(0.999),
                         eps_rel=f32(1e-8))
    b = wl["host"]
    a = b.Y.shape[0]
    cols = [int(q * a / n_sample) for q in range(n_sample)]
    Am = b.A
    As = W.bf16_values(b.At[:, :b.m]).astype(np.float64).T if wl["dtype"] == "bf16" else Am
    ys = [b.Y[c].astype(np.float64) for c in cols]

    def run_clomp():
        return [clomp_fp64(As, y, b.k, params, A_refine=Am) for y in ys]

    log(f"timing the FP64 oracle on {n_sample} columns (all threads, then one)")
    t0 = time.perf_counter()
    refs = run_clomp()
    t_all = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        run_clomp()
        t_one = time.perf_counter() - t0
    orefs = [omp_fp64(Am, y, b.k) for y in ys[:n_omp]]
    acc = {}
    for method, rr in (("clomp", refs), ("omp", orefs)):
        o = outs[method]
        rows = []
        for c, r, y in zip(cols, rr, ys):
            xs = o.x[c].cpu().numpy().astype(np.float64)
            rows.append((o.support[c][: int(o.n_selected[c])].cpu().tolist() == r.support,
                         float(np.linalg.norm(xs - r.x) / np.linalg.norm(r.x)),
                         float(np.linalg.norm(y - Am @ xs) / np.linalg.norm(y)),
                         float(np.linalg.norm(y - Am @ r.x) / np.linalg.norm(y))))
        same = [e for ok, e, _, _ in rows if ok]
        acc[method] = {"rel_err": max(same) if same else None,
                       "rel_err_median": float(np.median(same)) if same else None,
                       "rel_err_all_max": max(e for _, e, _, _ in rows),
                       "support_identical_fraction": len(same) / len(rows),
                       "resid_rel_median": float(np.median([g for _, _, g, _ in rows])),
                       "oracle_resid_rel_median": float(np.median([q for _, _, _, q in rows])),
                       "sample": f"{len(rows)} evenly spaced columns of {a}; rel_err over the "
                                 "columns whose ordered support equals the oracle's; "
                                 "resid_rel = ||y - A x|| / ||y|| (float32 A)"}
    cpu = {"value": len(cols) / t_all, "unit": "signals/s", "cores": _threads(), "kind": "oracle",
           "sample": f"{len(cols)} evenly spaced columns of the {a}, FP64 CLOMP oracle",
           "seconds": t_all, "host_cpus": os.cpu_count(),
           "one_core": {"value": len(cols) / t_one, "unit": "signals/s", "cores": 1,
                        "seconds": t_one}}
    return acc, cpu


if __name__ == "__main__":
    main()
