"""Benchmark: solves/s at n = 4096 to an FP64-level residual (<= 1e-13), mixed-precision
iterative refinement against the plain FP64 sign-function Newton solve, on one MI355X.

Workload (synthetic, seeded): n = 4096, W = L S L^T with L 4096 x 8 ~ N(0,1) and S = diag(+-1)
indefinite; A = Q T Q^T with Q Haar orthogonal and T upper triangular, diag(T) =
-logspace(-3, 0, n) (see lyapgen.config("large")).  Inputs are resident in HBM before timing.

One step = one complete lyap_solve call (inversions, factor iteration, residual
factorisations, corrections and updates) that must end with res <= 1e-13; a run whose solves
do not reach it is reported as DNF with its attained residual.  The plain FP64 solve and IR
with fp16, bf16 and fp32 inner solvers are timed; ``value`` is the IR with the fp16 inner
solver (the inner precision the workload names), the others are reported beside it: the
same paths with adaptive inner tolerances and with the butterfly inversion, the low-rank ADI
inner solver against FP64 ADI, and 256 independent equations of n in [64, 512] (a loop of
FP64 solves against the batched entry point).  The first timed solve of each path is
re-checked on the host: its residual (eq 4.1) recomputed in float64 NumPy from the returned
factors.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--inner fp16,bf16,fp32] [--adaptive fp16,fp32]
                  [--skip-cpu] [--skip-adi] [--skip-batched]
  python bench.py --traffic-run   (one IR solve and a calibration copy, for HBM counters)
  python bench.py --mfma-run [--us fp64]   (one solve and calibration products, for MFMA counters)
  python bench.py --inverse-run fp64:rbt   (three inversions, for kernel profiles)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp16": 2500.0, "bf16": 2500.0, "fp16x2": 2500.0}
PEAK_HBM_GBS = 8000.0


def _time_inverse(lyap, torch, A, us, reps=3, pivot=True):
    """Average duration of one inversion (2 n^3 flops) on the current stream, measured with
    HIP events around the calls."""
    lyap.inverse(A, us, pivot=pivot)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lyap.inverse(A, us, pivot=pivot)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def _batched(lyap, torch):
    """256 independent equations (n ~ U{64..512}, m ~ U{1..8}): a host loop of FP64 solves
    against the batched entry point (FP64, and IR with fp16 / fp32 inner solves, with fixed
    and adaptive inner tolerances).  One warm-up pass each."""
    import lyapgen

    batch = lyapgen.batch_family()
    As = [torch.from_numpy(a).cuda() for a, _ in batch]
    Ls = [torch.from_numpy(l).cuda() for _, l in batch]
    out = {}

    def loop():
        return [lyap.solve(a, l, None, precisions=("fp64",) * 4, raise_on_error=False)[2]
                for a, l in zip(As, Ls)]

    def batched(p, **opts):
        return [o[2] for o in lyap.solve_batched(As, Ls, None, precisions=p,
                                                 raise_on_error=False, **opts)]

    ir = ("fp64", "fp64", "fp64")
    for label, fn in (("loop_fp64", loop),
                      ("batched_fp64", lambda: batched(("fp64",) * 4)),
                      ("batched_fp16_ir", lambda: batched(("fp16",) + ir)),
                      ("batched_fp16_ir_adaptive", lambda: batched(("fp16",) + ir, adaptive=1)),
                      ("batched_fp32_ir", lambda: batched(("fp32",) + ir)),
                      ("batched_fp32_ir_adaptive", lambda: batched(("fp32",) + ir, adaptive=1))):
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
        print(f"batched {label}: {out[label]}", file=sys.stderr, flush=True)
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


def _inverse_run(lyap, torch, A, spec):
    """Untimed: three inversions of the n = 4096 matrix at ``dtype[:pivot]`` (pivot "partial",
    "none" or "rbt"), for per-kernel profiles of the inversion alone; then the calibration
    steps of the counter runs: one FP64, one FP32 and one FP16 library product of 4096^3
    (137.4 GFLOP each, the MFMA op counters' unit) and a plain copy of 256 MiB evicted from
    the MALL first (the HBM counters' scale)."""
    dt, _, pv = spec.partition(":")
    pivot = {"": True, "partial": True, "none": False, "rbt": "rbt"}[pv]
    for _ in range(3):
        lyap.inverse(A, dt, pivot=pivot)
    torch.cuda.synchronize()
    print("inversions done", dt, pv or "partial", flush=True)
    for t in (torch.float64, torch.float32, torch.float16):
        a = torch.ones((4096, 4096), dtype=t, device="cuda")
        c = torch.matmul(a, a)
        torch.cuda.synchronize()
        print("calibration matmul", t, "flops", 2 * 4096 ** 3, float(c[0, 0]), flush=True)
    x = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
    torch.cuda.synchronize()
    big = torch.empty(96 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(2.0)
    torch.cuda.synchronize()
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del big
    print("calibration copy bytes", x.numel() * 8, flush=True)


def _profile_value(name, key, hash_key, sources):
    """``key`` from the machine-readable tail of profiles/``name``, or None: the counters
    describe the code they were taken on, so the value is used only while the listed kernel
    sources (paper_2510_02126_amd/csrc) still have the recorded combined sha256."""
    import hashlib
    import re

    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            vals = dict(re.findall(r"^(\w+): (\S+)$", f.read(), re.M))
    except OSError:
        return None
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, "paper_2510_02126_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    if vals.get(hash_key) != h.hexdigest() or key not in vals:
        return None
    return float(vals[key])


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


def _host_relres(A, L, S, Z, D):
    """Relative residual of eq (4.1) for X = Z diag(D) Z^T, in float64 NumPy on the host from
    the factored form: R = F N F^T with F = [Z, AZ, L] and N = [[0, D, 0], [D, 0, 0],
    [0, 0, S]]; with the thin QR F = U T, ||R||_F = ||T N T^T||_F (no Gram matrix, so a
    residual near the rounding level is resolved).  ||X||_F = ||T_Z diag(D) T_Z^T||_F from
    the QR of Z alone."""
    import numpy as np

    r, m = Z.shape[1], L.shape[1]
    F = np.hstack([Z, A @ Z, L])
    T = np.linalg.qr(F, mode="r")
    N = np.zeros((2 * r + m, 2 * r + m))
    N[:r, r:2 * r] = np.diag(D)
    N[r:2 * r, :r] = np.diag(D)
    N[2 * r:, 2 * r:] = np.diag(S)
    normR = np.linalg.norm(T @ N @ T.T, "fro")
    Tz = np.linalg.qr(Z, mode="r")
    normX = np.linalg.norm((Tz * D[None, :]) @ Tz.T, "fro")
    Tl = np.linalg.qr(L, mode="r")
    normW = np.linalg.norm((Tl * S[None, :]) @ Tl.T, "fro")
    return normR / (normW + 2.0 * normX * np.linalg.norm(A, "fro"))


def _cpu_baseline(cfg):
    """The oracle's whole FP64 sign-function Newton solve (Alg 3.2 through the first residual
    evaluation, oracle.refine.ir_ldlt with refine=False) of the workload on the host cores."""
    from threadpoolctl import threadpool_info

    from oracle import refine as IR

    t0 = time.perf_counter()
    _, _, info = IR.ir_ldlt(cfg["A"], cfg["L"], cfg["S"], prec=("fp64",) * 4, refine=False)
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    return dt, threads, info


def _run_path(lyap, torch, cfg, A, L, S, us, steps, warmup, **opts):
    """Time ``steps`` solves of one path; the first timed solve is re-checked on the host."""
    prec = (us, "fp64", "fp64", "fp64")
    for _ in range(warmup):
        lyap.solve(A, L, S, precisions=prec, raise_on_error=False, **opts)
    torch.cuda.synchronize()
    infos, first = [], None
    t0 = time.perf_counter()
    for i in range(steps):
        Z, D, info = lyap.solve(A, L, S, precisions=prec, raise_on_error=False, **opts)
        infos.append(info)
        if i == 0:
            first = (Z, D)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    Zh, Dh = first[0].cpu().numpy(), first[1].cpu().numpy()
    host_res = _host_relres(cfg["A"], cfg["L"], cfg["S"], Zh, Dh)
    ok = all(i["status"] == "OK" and i["res"] <= 1e-13 for i in infos) and host_res <= 1e-13
    last = infos[-1]
    fam = {f: sum(i["kern_ms"][f] for i in infos) for f in range(4)}
    work = {f: sum(i["kern_work"][f] for i in infos) for f in range(4)}
    calls = {f: sum(i["kern_calls"][f] for i in infos) for f in range(4)}
    return {
        "us": us, "ok": ok, "dt": dt, "steps": steps, "infos": infos, "fam_ms": fam,
        "fam_work": work, "fam_calls": calls,
        "summary": {
            "status": "OK" if ok else "DNF",
            "solves_per_s": round(steps / dt, 4) if ok else 0.0,
            "ms_per_solve": round(1e3 * dt / steps, 2),
            "res": last["res"], "res_host_first": host_res, "rank": last["rank"],
            "refinements": last["refinements"],
            "iters": f'{last["newton_total"]}({last["newton_max"]})',
            "inversions": last["inversions"],
            "rbt_steps": last["rbt_steps"], "rbt_fallbacks": last["rbt_fallbacks"],
            "phase_ms": [round(x, 2) for x in last["phase_ms"]],
        },
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", default="fp16,bf16,fp32",
                    help="inner (solver) precisions of the IR runs; the first is the headline")
    ap.add_argument("--us", default=None, help="(untimed runs) solver precision")
    ap.add_argument("--adaptive", default="fp16,fp32",
                    help="inner precisions also timed with adaptive inexact inner tolerances")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-adi", action="store_true",
                    help="skip the low-rank ADI inner-solver comparison")
    ap.add_argument("--skip-batched", action="store_true",
                    help="skip the 256 independent equations, n in [64, 512] (batched mode)")
    ap.add_argument("--traffic-run", action="store_true",
                    help="one untimed IR solve and a calibration copy (for HBM counters)")
    ap.add_argument("--mfma-run", action="store_true",
                    help="one untimed solve and calibration products (for MFMA counters)")
    ap.add_argument("--inverse-run", default=None, metavar="DTYPE[:PIVOT]",
                    help="three untimed inversions of the workload matrix (for kernel profiles)")
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
        _traffic_run(lyap, torch, A, L, S, args.us or "fp32")
        return
    if args.mfma_run:
        _mfma_run(lyap, torch, A, L, S, args.us or "fp32")
        return
    if args.inverse_run:
        _inverse_run(lyap, torch, A, args.inverse_run)
        return

    inner = [x.strip() for x in args.inner.split(",") if x.strip()]
    base = _run_path(lyap, torch, cfg, A, L, S, "fp64", args.steps, args.warmup)
    print(f"fp64: {base['summary']}", file=sys.stderr, flush=True)
    runs = {}
    for us in inner:
        # bf16 solves take many refinements at this condition number: one timed solve
        st, wu = (1, 0) if us == "bf16" else (args.steps, args.warmup)
        runs[us] = _run_path(lyap, torch, cfg, A, L, S, us, st, wu)
        print(f"ir {us}: {runs[us]['summary']}", file=sys.stderr, flush=True)
    adaptive, fast = {}, {}
    for us in [x.strip() for x in args.adaptive.split(",") if x.strip()]:
        adaptive[us] = _run_path(lyap, torch, cfg, A, L, S, us, args.steps, args.warmup,
                                 adaptive=1)
        print(f"ir {us} adaptive: {adaptive[us]['summary']}", file=sys.stderr, flush=True)
    # the same paths with the random butterfly transformation in place of partial pivoting
    base_rbt = _run_path(lyap, torch, cfg, A, L, S, "fp64", args.steps, args.warmup, pivoting=1)
    print(f"fp64 rbt: {base_rbt['summary']}", file=sys.stderr, flush=True)
    for us in [x.strip() for x in args.adaptive.split(",") if x.strip()]:
        fast[us] = _run_path(lyap, torch, cfg, A, L, S, us, args.steps, args.warmup, adaptive=1,
                             pivoting=1)
        print(f"ir {us} adaptive rbt: {fast[us]['summary']}", file=sys.stderr, flush=True)
    # the second inner solver (low-rank ADI): FP64 ADI against IR with an fp32 ADI inner solve,
    # both with butterfly inversions
    adi = None
    if not args.skip_adi:
        adi64 = _run_path(lyap, torch, cfg, A, L, S, "fp64", args.steps, args.warmup, solver=1,
                          pivoting=1)
        print(f"adi fp64 rbt: {adi64['summary']}", file=sys.stderr, flush=True)
        adi32 = _run_path(lyap, torch, cfg, A, L, S, "fp32", args.steps, args.warmup, solver=1,
                          pivoting=1, adaptive=1)
        print(f"adi ir fp32 adaptive rbt: {adi32['summary']}", file=sys.stderr, flush=True)
        a64 = adi64["summary"]["solves_per_s"]
        adi = {"fp64_adi_rbt": adi64["summary"],
               "ir_fp32_adi_adaptive_rbt": dict(
                   adi32["summary"],
                   speedup_vs_fp64_adi=(round(adi32["summary"]["solves_per_s"] / a64, 4)
                                        if adi64["ok"] and adi32["ok"] else None))}
    head = runs[inner[0]] if inner else base
    sps64 = base["summary"]["solves_per_s"]

    # roofline of the inversion (A2, 2 n^3 flops each; the matrix-core-bound step) in the
    # headline IR solves, from the library's HIP-event accounting on the solve's stream
    peak = PEAK_TFLOPS[head["us"]]
    inv_ms, inv_flops, inv_calls = head["fam_ms"][0], head["fam_work"][0], head["fam_calls"][0]
    achieved = inv_flops / (inv_ms * 1e-3) / 1e12 if inv_ms > 0 else 0.0
    roof = {"bound": "mfma", "kernel": "inversion (Gauss-Jordan: pivoted leaves + MFMA block "
            f"updates), {head['us']} operands, 2 n^3 flops per inversion",
            "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 5),
            "traffic": (_profile_value("inversion_fp16_n4096_hbm_traffic.md",
                                       "traffic_bytes_per_inversion", "sources_sha256",
                                       ["inverse.hip", "gemm.hip"])
                        if head["us"] == "fp16" else None),
            "launches": inv_calls, "avg_launch_us": round(1e3 * inv_ms / max(1, inv_calls), 1)}
    total_ms = 1e3 * head["dt"]
    shares = {
        "inversion": round(head["fam_ms"][0] / total_ms, 4),
        "jacobi_rounds (spectral decompositions, latency-bound)": round(head["fam_ms"][1] / total_ms, 4),
        "thin_qr (latency-bound panels + MFMA updates)": round(head["fam_ms"][2] / total_ms, 4),
    }
    shares["rest (products, norms, copies, host)"] = round(1.0 - sum(shares.values()), 4)
    jac = {"achieved_GBs": round(head["fam_work"][1] / (head["fam_ms"][1] * 1e-3) / 1e9, 1)
           if head["fam_ms"][1] > 0 else None, "peak_GBs": PEAK_HBM_GBS,
           "launches": head["fam_calls"][1],
           "traffic_bytes_per_launch_fp32_ir": _profile_value(
               "jac_round_n4096_ir_fp32_hbm_traffic.md", "traffic_bytes_per_launch",
               "eig_hip_sha256", ["eig.hip"])}
    t_inv = _time_inverse(lyap, torch, A, "fp64")
    inv64 = 2.0 * n ** 3 / t_inv / 1e12
    t_inv_rbt = _time_inverse(lyap, torch, A, "fp64", pivot="rbt")
    inv64_rbt = 2.0 * n ** 3 / t_inv_rbt / 1e12

    batched = None if args.skip_batched else _batched(lyap, torch)

    cpu = None
    if not args.skip_cpu:
        dt_cpu, threads, cinfo = _cpu_baseline(cfg)
        cpu = {"value": round(1.0 / dt_cpu, 6), "unit": "solves/s", "cores": threads,
               "kind": "oracle",
               "sample": f"one whole oracle FP64 sign-function Newton solve of the n={n} workload "
                         f"(Alg 3.2, K={cinfo.inversions}, first residual evaluated; "
                         f"{dt_cpu:.1f} s on the host cores)"}

    line = {
        "metric": "solves/s at n=4096 to FP64-level residual: mixed-prec IR vs FP64 sign-Newton",
        "value": head["summary"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * head["dt"] / head["steps"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{head['us']}-inner/f64",
        "data": "synthetic",
        "config": {"workload": "n=4096, m=8, W=L S L^T indefinite, A=Q T Q^T kappa~1e3",
                   "ir_precisions": [head["us"], "fp64", "fp64", "fp64"], "tol": 1e-13},
        "ir": {us: r["summary"] for us, r in runs.items()},
        "fp64_sign_newton": base["summary"],
        "speedup_vs_fp64": {us: (round(r["summary"]["solves_per_s"] / sps64, 4)
                                 if sps64 > 0 and r["ok"] else None) for us, r in runs.items()},
        "ir_adaptive_inner_tolerances": {
            us: dict(r["summary"], speedup_vs_fp64=(round(r["summary"]["solves_per_s"] / sps64, 4)
                                                    if sps64 > 0 and r["ok"] else None))
            for us, r in adaptive.items()},
        "fp64_sign_newton_rbt": base_rbt["summary"],
        "low_rank_adi": adi,
        "ir_adaptive_rbt": {
            us: dict(r["summary"], speedup_vs_fp64_rbt=(
                round(r["summary"]["solves_per_s"] / base_rbt["summary"]["solves_per_s"], 4)
                if base_rbt["ok"] and r["ok"] else None))
            for us, r in fast.items()},
        "roofline": roof,
        "time_shares_headline_ir": shares,
        "jacobi_rounds_hbm": jac,
        "inversion_fp64_alone": {"ms": round(1e3 * t_inv, 3), "tflops": round(inv64, 3),
                                 "frac_fp64_peak": round(inv64 / PEAK_TFLOPS["fp64"], 4)},
        "inversion_fp64_rbt_alone": {"ms": round(1e3 * t_inv_rbt, 3),
                                     "tflops": round(inv64_rbt, 3),
                                     "frac_fp64_peak": round(inv64_rbt / PEAK_TFLOPS["fp64"], 4)},
        "cpu_baseline": cpu,
    }
    if batched is not None:
        line["batched_256_n64_512"] = batched
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
