"""Benchmark: solves/s at n = 4096 to an FP64-level residual (<= 1e-13), mixed-precision
iterative refinement against the plain FP64 sign-function Newton solve, on one MI355X.

Workload (synthetic, seeded): n = 4096, W = L S L^T with L 4096 x 8 ~ N(0,1) and S = diag(+-1)
indefinite; A = Q T Q^T with Q Haar orthogonal and T upper triangular, diag(T) =
-logspace(-3, 0, n) (see lyapgen.config("large")).  Inputs are resident in HBM before timing.

One step = one complete lyap_solve call (inversions, factor iteration, residual
factorisations, corrections and updates) that must end with res <= 1e-13; a run whose solves
do not reach it is reported as DNF.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--us fp32] [--skip-cpu] [--batched]
  python bench.py --traffic-run   (one IR solve and a calibration copy, for HBM counters)
  python bench.py --mfma-run [--us fp64]   (one solve and calibration products, for MFMA counters)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp16": 2500.0, "bf16": 2500.0}
PEAK_HBM_GBS = 8000.0


def _time_solves(lyap, torch, A, L, S, us, steps, warmup):
    for _ in range(warmup):
        lyap.solve(A, L, S, precisions=(us, "fp64", "fp64", "fp64"), raise_on_error=False)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, info = lyap.solve(A, L, S, precisions=(us, "fp64", "fp64", "fp64"),
                                raise_on_error=False)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, infos


def _time_inverse(lyap, torch, A, us, reps=3):
    """Average duration of one inversion (the dominant kernel family, 2 n^3 flops) on the
    current stream, measured with HIP events around the calls."""
    lyap.inverse(A, us)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lyap.inverse(A, us)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def _batched(lyap, torch, us):
    """256 independent equations (n ~ U{64..512}, m ~ U{1..8}): a host loop of FP64 solves
    against the batched entry point (FP64 and IR at ``us``).  One warm-up pass each."""
    import lyapgen

    batch = lyapgen.batch_family()
    As = [torch.from_numpy(a).cuda() for a, _ in batch]
    Ls = [torch.from_numpy(l).cuda() for _, l in batch]
    out = {}

    def loop():
        return [lyap.solve(a, l, None, precisions=("fp64",) * 4, raise_on_error=False)[2]
                for a, l in zip(As, Ls)]

    def batched(p):
        return [o[2] for o in lyap.solve_batched(As, Ls, None, precisions=p,
                                                 raise_on_error=False)]

    for label, fn in (("loop_fp64", loop),
                      ("batched_fp64", lambda: batched(("fp64",) * 4)),
                      (f"batched_{us}_ir", lambda: batched((us, "fp64", "fp64", "fp64")))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = all(i["status"] == "OK" and i["res"] <= 1e-13 for i in infos)
        out[label] = {"solves_per_s": round(len(infos) / dt, 2) if ok else 0.0,
                      "max_res": max(i["res"] for i in infos),
                      "status": "OK" if ok else "DNF"}
    return out


def _traffic_run(lyap, torch, A, L, S, us):
    """Untimed: one IR solve, then a plain copy of known size for scaling the HBM counters
    (a 256 MiB float64 tensor, evicted from the MALL by writing 768 MiB of other data, copied
    once).  Run under ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``."""
    _, _, info = lyap.solve(A, L, S, precisions=(us, "fp64", "fp64", "fp64"),
                            raise_on_error=False)
    torch.cuda.synchronize()
    print("ir", info["status"], info["res"], "jac_round launches", info["kern_calls"][1],
          "algorithmic bytes", info["kern_work"][1], flush=True)
    x = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
    torch.cuda.synchronize()
    big = torch.empty(96 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(2.0)
    torch.cuda.synchronize()
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del big
    print("calibration copy bytes", x.numel() * 8, flush=True)


def _mfma_run(lyap, torch, A, L, S, us):
    """Untimed: one solve at inner precision ``us``, then one FP64 and one FP32 product of
    4096^3 (torch.matmul, 137.4 GFLOP each) whose MFMA op counters give the counters' unit.
    Run under ``rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_F32 ...
    --kernel-trace``."""
    _, _, info = lyap.solve(A, L, S, precisions=(us, "fp64", "fp64", "fp64"),
                            raise_on_error=False)
    torch.cuda.synchronize()
    print("solve", us, info["status"], info["res"], "inversion flops", info["kern_work"][0],
          "inversions", info["kern_calls"][0], flush=True)
    for dt in (torch.float64, torch.float32):
        a = torch.ones((4096, 4096), dtype=dt, device="cuda")
        c = torch.matmul(a, a)
        torch.cuda.synchronize()
        print("calibration matmul", dt, "flops", 2 * 4096 ** 3, float(c[0, 0]), flush=True)


def _measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when there is none or the kernel's source changed since it was taken."""
    import hashlib
    import re

    if kernel != "jac_round":
        return None
    path = os.path.join(ROOT, "profiles", "jac_round_n4096_ir_fp32_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2510_02126_amd", "csrc", "eig.hip")
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    h = re.search(r"^eig_hip_sha256: ([0-9a-f]+)", text, re.M)
    if not t or not h or h.group(1) != digest:
        return None
    return float(t.group(1))


def _cpu_baseline(cfg, steps=6):
    """The oracle's FP64 sign-function Newton solve (Alg 3.2) on the host cores, on a bounded
    sample: its first ``steps`` Newton steps (inversion, scaled update, factor product), scaled
    to the full solve by K / steps with the Newton count K taken from the GPU run."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import signnewton as SN

    A, L = cfg["A"], cfg["L"]
    t0 = time.perf_counter()
    # ``steps`` Newton steps through the oracle's own routines
    Ak = A.copy()
    Z = L.copy()
    for _ in range(steps):
        Ainv = SN.inverse_at(Ak, "fp64")
        mu = float(np.sqrt(np.linalg.norm(Ainv, "fro") / np.linalg.norm(Ak, "fro")))
        Ak = 0.5 * (mu * Ak + Ainv / mu)
        Z = np.hstack([Z, Ainv @ Z])
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    return dt / steps, threads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--us", default="fp32", help="solver precision of the IR run")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="also time 256 independent equations, n in [64, 512] (batched mode)")
    ap.add_argument("--traffic-run", action="store_true",
                    help="one untimed IR solve and a calibration copy (for HBM counters)")
    ap.add_argument("--mfma-run", action="store_true",
                    help="one untimed solve and calibration products (for MFMA counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path; --gpus must be 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lyapgen
    import paper_2510_02126_amd as lyap

    cfg = lyapgen.config("large")
    A = torch.from_numpy(cfg["A"]).cuda()
    L = torch.from_numpy(cfg["L"]).cuda()
    S = torch.from_numpy(cfg["S"]).cuda()
    n = A.shape[0]
    if args.traffic_run:
        _traffic_run(lyap, torch, A, L, S, args.us)
        return
    if args.mfma_run:
        _mfma_run(lyap, torch, A, L, S, args.us)
        return

    # plain FP64 sign-function Newton solve (the baseline), then mixed-precision IR
    dt64, inf64 = _time_solves(lyap, torch, A, L, S, "fp64", args.steps, args.warmup)
    dtir, infir = _time_solves(lyap, torch, A, L, S, args.us, args.steps, args.warmup)
    ok64 = all(i["status"] == "OK" and i["res"] <= 1e-13 for i in inf64)
    okir = all(i["status"] == "OK" and i["res"] <= 1e-13 for i in infir)
    sps64 = args.steps / dt64 if ok64 else 0.0
    spsir = args.steps / dtir if okir else 0.0

    # roofline of the dominant kernel family of the timed IR solves, from the HIP-event
    # accounting the library keeps per solve (summed over the timed solves)
    fam_ms = [sum(i["kern_ms"][f] for i in infir) for f in range(4)]
    fam_work = [sum(i["kern_work"][f] for i in infir) for f in range(4)]
    fam_calls = [sum(i["kern_calls"][f] for i in infir) for f in range(4)]
    fams = {
        0: ("inversion (Gauss-Jordan leaves + MFMA block updates, 2n^3 flops)", "mfma",
            "TFLOP/s", 1e12, PEAK_TFLOPS["fp32" if args.us == "fp32" else args.us]),
        1: ("jac_round (Jacobi round: block rotation update of A and V, ~24 pp^2 bytes)",
            "hbm", "GB/s", 1e9, PEAK_HBM_GBS),
        2: ("thin QR (Householder TSQR panels + compact-WY MFMA updates)", "mfma", "TFLOP/s",
            1e12, PEAK_TFLOPS["fp64"]),
    }
    dom = max(fams, key=lambda f: fam_ms[f])
    name, bound, unit, scale, peak = fams[dom]
    achieved = fam_work[dom] / (fam_ms[dom] * 1e-3) / scale if fam_ms[dom] > 0 else 0.0
    traffic = _measured_traffic(name.split(" ")[0])
    roof = {"bound": bound, "kernel": name, "achieved": round(achieved, 3), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4), "traffic": traffic,
            "launches": fam_calls[dom], "avg_launch_us": round(1e3 * fam_ms[dom] /
                                                                max(1, fam_calls[dom]), 2)}
    breakdown = {}
    for f, (nm, bd, un, sc, pk) in fams.items():
        if fam_ms[f] > 0:
            ach = fam_work[f] / (fam_ms[f] * 1e-3) / sc
            breakdown[nm.split(" ")[0]] = {"ms_per_solve": round(fam_ms[f] / args.steps, 2),
                                           "achieved": round(ach, 3), "unit": un,
                                           "frac": round(ach / pk, 4)}
    t_inv = _time_inverse(lyap, torch, A, "fp64")
    inv64 = 2.0 * n ** 3 / t_inv / 1e12

    batched = _batched(lyap, torch, args.us) if args.batched else None

    cpu = None
    if not args.skip_cpu:
        K = inf64[-1]["inversions"]
        steps_cpu = max(1, min(6, K))
        t_step, threads = _cpu_baseline(cfg, steps_cpu)
        t_solve = t_step * K
        cpu = {"value": round(1.0 / t_solve, 6), "unit": "solves/s", "cores": threads,
               "kind": "oracle",
               "sample": f"oracle FP64 sign-Newton, first {steps_cpu} of K={K} Newton steps at "
                         f"n={n} ({steps_cpu * t_step:.1f} s), scaled to a full solve"}

    line = {
        "metric": "solves/s at n=4096 to FP64-level residual: mixed-prec IR vs FP64 sign-Newton",
        "value": round(spsir, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dtir / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.us}-inner/f64",
        "data": "synthetic",
        "config": {"workload": "n=4096, m=8, W=L S L^T indefinite, A=Q T Q^T kappa~1e3",
                   "ir_precisions": [args.us, "fp64", "fp64", "fp64"], "tol": 1e-13},
        "ir": {"solves_per_s": round(spsir, 4), "res": infir[-1]["res"],
               "rank": infir[-1]["rank"], "refinements": infir[-1]["refinements"],
               "iters": f'{infir[-1]["newton_total"]}({infir[-1]["newton_max"]})',
               "phase_ms": [round(x, 2) for x in infir[-1]["phase_ms"]],
               "status": "OK" if okir else "DNF"},
        "fp64_sign_newton": {"solves_per_s": round(sps64, 4),
                             "ms_per_solve": round(1e3 * dt64 / args.steps, 3),
                             "res": inf64[-1]["res"], "rank": inf64[-1]["rank"],
                             "K": inf64[-1]["inversions"],
                             "phase_ms": [round(x, 2) for x in inf64[-1]["phase_ms"]],
                             "status": "OK" if ok64 else "DNF"},
        "speedup_ir_vs_fp64": round(spsir / sps64, 4) if sps64 > 0 and spsir > 0 else None,
        "roofline": roof,
        "kernel_families_ir": breakdown,
        "inversion_fp64_alone": {"ms": round(1e3 * t_inv, 3), "tflops": round(inv64, 3),
                                 "frac_fp64_peak": round(inv64 / PEAK_TFLOPS["fp64"], 4)},
        "cpu_baseline": cpu,
    }
    if batched is not None:
        line["batched_256_n64_512"] = batched
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
