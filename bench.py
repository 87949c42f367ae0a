#!/usr/bin/env python3
"""Throughput of the ETDM energy+gradient path on one MI355X.

One "step" is one evaluation of E and the full gradient for every instance of
the workload (all steps of the hot path).  The default workload is the largest
single-GPU one: the 576-water box (M = 13248, N = 2304, block-sparse H0) in the
mixed mode (P = B B^T, V = X^T B and the eigensolver in FP64, the bulk
contractions as 3-way BF16 splits on the matrix cores), with full L-BFGS iterations
timed beside it.  Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line (rank 0, N = 1):
  value            evaluations per second (whole job)
  roofline         dominant stage: algorithmic flops (or bytes) per launch over its
                   average HIP-event duration in the timed region, vs MI355X peak
  roofline_end_to_end, roofline_gemm_phase
                   T_roofline / T_measured with T_roofline = sum over stages of
                   max(flops / peak of the stage's arithmetic, bytes / HBM peak)
  cpu_baseline     the FP64 oracle (structured ov path for the real workloads) on the
                   host cores, with the CPU model and the thread count
  parity           |dE| per electron, relative |dg| and element-wise max |dg| / max |g|
                   of this run vs the oracle
  fp64_path        the same kernels in FP64 mode, and the speedup over it
  lbfgs            full L-BFGS iterations (direction, line search, memory update)

--cpu-only times the oracle alone (no GPU work), e.g. with --cpu-threads 1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ETDM energy+gradient evals/sec, MFMA TFLOP/s vs peak, at stated |dE|"
# MI355X dense peaks (TFLOP/s); a p-product BF16 split does 1/p of the BF16 rate in
# useful flops
FP64_PEAK = 78.6
SPLIT_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3, "bf16x6": 2500.0 / 6,
                     "mixed": 2500.0 / 6}
HBM_PEAK_GBS = 8000.0
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16", "mixed": "f64+bf16x6"}
WORKLOADS = {
    1: "config 1: chain Hamiltonian M=64 N=16, real, one molecule",
    2: "config 2: 148 ragged G2-like molecules, M~U[20,400], N=round(M/5), real, Hubbard U=0.5",
    3: "config 3: 64-water box M=1472 N=256, block-sparse H0, real",
    4: "config 4: crystal 4x4x4 k-grid, M=208, complex, Fermi-Dirac f, k-coupled Hubbard",
    5: "config 5: 576-water box M=13248 N=2304, block-sparse H0, real",
}
DEFAULT_PREC = {1: "fp64", 2: "mixed", 3: "mixed", 4: "mixed", 5: "mixed"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-only", action="store_true", help="time the oracle only (no GPU work)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="BLAS threads of the oracle (0: all)")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the oracle (parity and CPU baseline), e.g. for profiling runs")
    ap.add_argument("--lbfgs-iters", type=int, default=None,
                    help="also time this many L-BFGS iterations (default 3 on config 5, else 0)")
    ap.add_argument("--lbfgs-reset-norm", type=float, default=0.0,
                    help="L-BFGS: also reset the reference orbitals when an instance's |A| exceeds this")
    ap.add_argument("--gemm-tuning", type=int, default=0, choices=range(7),
                    help="GEMM kernel choice: 0 tuned at creation, 1 size rule, 2 packed 128x128, "
                         "3 grouped 64x64, 4 packed 64x64, 5 packed 128x64, 6 packed 64x128")
    ap.add_argument("--expm", default="eig", choices=("eig", "ss"),
                    help="exp(A) through eigh(iA) (Eq. ed) or scaling and squaring with a Pade "
                         "approximant (Eq. ss; complex workloads with --gradient approx)")
    ap.add_argument("--overlap", action="store_true",
                    help="the workload in a non-orthogonal basis (dense-H0 workloads)")
    ap.add_argument("--odd-lambda", type=float, default=0.0,
                    help="strength of the orbital-dependent model term (complex workloads)")
    ap.add_argument("--gradient", default="exact", choices=("exact", "approx"),
                    help="exact dE/dA (Eq. gradients) or the approximation G ~ L^T (Eq. app_grad)")
    return ap.parse_args()


def build_handle(wl, precision, gemm_tuning=0, gradient="exact", expm="eig", odd_lambda=0.0):
    import torch
    from paper_2101_12597_amd import Handle
    from workloads.pack import pack
    pk = pack(wl, use_bsr=wl.instances[0].H0_bsr is not None)
    dev = torch.device("cuda:0")
    H0 = torch.from_numpy(pk["H0"]).to(dev)
    C0 = torch.from_numpy(pk["C0"]).to(dev)
    S = torch.from_numpy(pk["S"]).to(dev) if pk.get("S") is not None else None
    h = Handle(pk["M"], pk["N"], wl.kind, precision, wl.hubbard_U, H0, C0, pk["f"],
               couple=wl.couple, weights=pk["weights"], bsr=pk["bsr"], gemm_tuning=gemm_tuning,
               gradient=gradient, expm=expm, odd_lambda=odd_lambda, overlap=S)
    A = torch.from_numpy(pk["A"]).to(dev)
    E = torch.empty(h.n_inst + 1, dtype=torch.float64, device=dev)
    G = torch.empty_like(A)
    del H0, C0, S
    torch.cuda.synchronize()
    return h, A, E, G


def timed_run(h, A, E, G, steps, warmup, time_stage=None):
    import torch
    for _ in range(warmup):
        h.energy_grad(A, E, G)
    h.sync_status()
    if time_stage is not None:
        h.reset_timing()
        h.set_timing(1 << time_stage)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.energy_grad(A, E, G)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.sync_status()
    stages = h.stage_info() if time_stage is not None else None
    h.set_timing(0)
    return (t1 - t0) / steps, stages


def stage_profile(h, A, E, G, reps=5):
    """Per-stage HIP-event times over a few evaluations (all stages timed)."""
    import torch
    h.reset_timing()
    h.set_timing(-1)
    for _ in range(reps):
        h.energy_grad(A, E, G)
    torch.cuda.synchronize()
    info = h.stage_info()
    h.set_timing(0)
    h.reset_timing()
    return info


def gemm_kernel_table(h, prof):
    """Kernel of every GEMM stage; for the FP64 / BF16x6 stages also the launch times
    (ms) of the three kernels measured by the tuning at handle creation."""
    names = {r["index"]: r["name"] for r in prof}
    out = {}
    for k in h.stage_kernels():
        if not k["kernel"]:
            continue
        entry = {"kernel": k["kernel"]}
        if any(v > 0 for v in k["tuned_ms"].values()):
            entry["tuned_ms"] = {n: round(v, 4) for n, v in k["tuned_ms"].items()}
        out[names.get(k["index"], str(k["index"]))] = entry
    return out


def oracle_reference(wl, params, gradient="exact", expm="eig", odd_lambda=0.0, progress=None):
    """Per-instance E and g from the FP64 oracle, its wall time and its route.  Real
    workloads in an orthonormal basis take the structured occupied-virtual path (the
    oracle the CPU baseline times; the GPU tests pin it to the definition path);
    complex workloads, k-coupled densities and non-orthogonal bases take the
    definition path (the eigendecomposition of iA)."""
    import copy
    import numpy as np
    from oracle import etdm as O
    t0 = time.perf_counter()
    Es, gs = [], []
    if wl.kind == "real_ov" and not wl.couple and all(i.S is None for i in wl.instances) and odd_lambda == 0.0:
        for inst, p in zip(wl.instances, params):
            if gradient == "exact":
                e, g = O.energy_grad_ov(inst, p, wl.hubbard_U, progress=progress)
            else:
                e, g = O.energy_grad_ov_approx(inst, p, wl.hubbard_U)
            Es.append(e)
            gs.append(g)
            if progress:
                progress(f"oracle instance {len(Es)}/{len(wl.instances)} done")
        return np.array(Es), gs, time.perf_counter() - t0, "structured occupied-virtual path"
    route = "definition path (eigendecomposition of iA)"
    if odd_lambda != 0.0:  # the orbital-dependent term (complex workloads, exact gradient)
        e, gs = O.energy_grad_odd(wl, params, odd_lambda)
        return np.array([e]), gs, time.perf_counter() - t0, route
    if wl.couple:
        if gradient == "exact":
            e, gs = O.energy_grad(wl, params)
        else:
            e, gs = O.energy_grad_approx(wl, params, expm=O.expm_ss if expm == "ss" else None)
        return np.array([e]), gs, time.perf_counter() - t0, route
    for inst, p in zip(wl.instances, params):
        sub = copy.copy(wl)
        sub.instances = [inst]
        if gradient == "exact":
            e, (g,) = O.energy_grad(sub, [p])
        else:
            e, (g,) = O.energy_grad_approx(sub, [p], expm=O.expm_ss if expm == "ss" else None)
        Es.append(e)
        gs.append(g)
    return np.array(Es), gs, time.perf_counter() - t0, route


def measured_traffic(stage, cfg, prec):
    """HBM bytes per launch of `stage` from a committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (profiles/*_traffic_pmc.txt, copy-calibrated), or None when there is none
    for this workload or the kernel source changed since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic_pmc.txt")):
        for line in open(path):
            if not line.startswith("# traffic:"):
                continue
            kv = dict(tok.split("=", 1) for tok in line[len("# traffic:"):].split())
            if kv.get("stage") != stage or kv.get("config") != str(cfg) or kv.get("precision") != prec:
                continue
            # source: the kernel's files, comma-separated, hashed in that order
            h = hashlib.sha256()
            for rel in kv["source"].split(","):
                src = os.path.join(ROOT, rel)
                if not os.path.exists(src):
                    return None
                h.update(open(src, "rb").read())
            if h.hexdigest()[:16] != kv["sha256"]:
                return None
            return float(kv["bytes_per_launch"])
    return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else os.cpu_count()
    except Exception:
        return os.cpu_count()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def blas_limit(threads):
    """Context limiting the BLAS pool of the oracle (threads = 0: leave it)."""
    import contextlib
    if threads <= 0:
        return contextlib.nullcontext()
    from threadpoolctl import threadpool_limits
    return threadpool_limits(limits=threads, user_api="blas")


def stage_peak_tflops(kernel, name, prec):
    """Peak of the arithmetic a stage runs in: its GEMM kernel's (FP64 kernels and the
    complex FP64 GEMM at the FP64 MFMA rate, the split kernels at BF16 / p), FP64 for
    the eigensolvers, None for the elementwise stages (bound by HBM)."""
    if kernel:
        if kernel.startswith(("fp64_", "zgemm")):
            return FP64_PEAK
        return SPLIT_PEAK_TFLOPS[prec]
    if name.startswith("eigh") or name in ("z_eigh", "ss_solve"):
        return FP64_PEAK
    return None


def roofline_fractions(prof, kernels, prec, ms_per_step):
    """End-to-end and GEMM-phase roofline fractions T_roofline / T_measured, with
    T_roofline = sum over the stages of one evaluation of max(flops / peak, bytes / HBM)
    and the stages' own HIP-event times for the GEMM phase."""
    by_index = {k["index"]: k["kernel"] for k in kernels}
    t_all = t_gemm = meas_gemm = 0.0
    for r in prof:
        if not r["launches"]:
            continue
        kern = by_index.get(r["index"], "")
        peak = stage_peak_tflops(kern, r["name"], prec)
        t_flop = r["flops"] / (peak * 1e12) if peak else 0.0
        t = max(t_flop, r["bytes"] / (HBM_PEAK_GBS * 1e9)) * 1e3
        t_all += t
        if kern:
            t_gemm += t
            meas_gemm += r["total_ms"] / r["launches"]
    return ({"t_roofline_ms": t_all, "t_measured_ms": ms_per_step, "frac": t_all / ms_per_step},
            {"t_roofline_ms": t_gemm, "t_measured_ms": meas_gemm,
             "frac": t_gemm / meas_gemm if meas_gemm > 0 else None})


def cpu_only(args):
    """Times the oracle alone: warm-up evaluations, then the median of --steps."""
    import numpy as np
    from oracle import etdm as O
    from workloads import make_config
    cfg = args.config
    log(f"generating config {cfg}")
    wl = make_config(cfg)
    params = O.parity_params(wl)
    times = []
    with blas_limit(args.cpu_threads):
        threads = blas_threads()
        for k in range(args.warmup + args.steps):
            _, _, t, route = oracle_reference(wl, params, args.gradient, args.expm, args.odd_lambda, progress=log)
            log(f"evaluation {k + 1}: {t:.2f} s")
            if k >= args.warmup:
                times.append(t)
    med = float(np.median(times))
    print(json.dumps({"metric": "oracle evaluations/s", "value": 1.0 / med, "unit": "evals/s",
                      "median_s": med, "times_s": times, "threads": threads, "cpu_model": cpu_model(),
                      "route": route, "config": {"workload": WORKLOADS[cfg]}, "warmup": args.warmup}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}): the path is a "
              "single-device one; sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.cpu_only:
        cpu_only(args)
        return
    import numpy as np
    import torch
    from oracle import etdm as O  # only for the parity numbers and the CPU baseline leg
    from workloads import make_config
    from workloads.pack import unpack_params

    cfg = args.config
    prec = args.precision or DEFAULT_PREC[cfg]
    lbfgs_iters = args.lbfgs_iters if args.lbfgs_iters is not None else (3 if cfg == 5 else 0)
    log(f"generating config {cfg}")
    wl = make_config(cfg)
    if args.overlap:
        from workloads import with_overlap
        wl = with_overlap(wl)
    params = O.parity_params(wl)
    log("creating the handle")
    t_create = time.perf_counter()
    h, A, E, G = build_handle(wl, prec, args.gemm_tuning, args.gradient, args.expm, args.odd_lambda)
    t_create = time.perf_counter() - t_create
    log("stage profile")

    # which stage dominates: time every stage over a few evaluations
    for _ in range(max(1, args.warmup)):
        h.energy_grad(A, E, G)
    h.sync_status()
    prof = stage_profile(h, A, E, G)
    dom = max(prof, key=lambda r: r["total_ms"])
    kernels = h.stage_kernels()

    log(f"dominant stage {dom['name']}; timed runs")
    # throughput: the launch sequence replayed from a captured HIP graph
    h.set_graph(True)
    sec, _ = timed_run(h, A, E, G, args.steps, args.warmup)
    h.set_graph(False)
    # dominant stage: HIP events around its launches over a timed region of the same
    # length (eager launches; the kernels are the same as in the graph)
    sec_eager, stages = timed_run(h, A, E, G, args.steps, args.warmup, time_stage=dom["index"])
    dstage = stages[dom["index"]]
    avg_ms = dstage["total_ms"] / max(dstage["launches"], 1)
    total_flops = sum(r["flops"] for r in prof)

    # parity of this run against the FP64 oracle at the same inputs
    h.energy_grad(A, E, G)
    h.sync_status()
    E_gpu = E.cpu().numpy()
    g_gpu = unpack_params(wl, G.cpu().numpy())
    if args.no_parity:
        dE = dg = de = None
        route = None
        args.no_cpu_baseline = True
    else:
        log("oracle reference")
        with blas_limit(args.cpu_threads):
            oracle_threads = blas_threads()
            Es, gs, t_oracle, route = oracle_reference(wl, params, args.gradient, args.expm, args.odd_lambda,
                                                       progress=log if cfg == 5 else None)
    if args.no_parity:
        pass
    elif wl.couple or len(Es) == 1 and len(wl.instances) > 1:
        dE = abs(E_gpu[-1] - Es[0]) / wl.n_electrons
        g_all, r_all = np.concatenate([x.ravel() for x in g_gpu]), np.concatenate([x.ravel() for x in gs])
        dg = float(np.linalg.norm(g_all - r_all) / np.linalg.norm(r_all))
        de = float(np.abs(g_all - r_all).max() / np.abs(r_all).max())
    else:
        dE = max(abs(E_gpu[k] - Es[k]) / max(inst.f.sum(), 1.0) for k, inst in enumerate(wl.instances))
        dg = max(float(np.linalg.norm(g_gpu[k] - gs[k]) / max(np.linalg.norm(gs[k]), 1e-300))
                 for k in range(len(wl.instances)))
        de = max((float(np.abs(g_gpu[k] - gs[k]).max() / max(np.abs(gs[k]).max(), 1e-300))
                  for k in range(len(wl.instances)) if gs[k].size), default=0.0)

    # dominant stage against the peak of its own arithmetic
    kern = {k["index"]: k["kernel"] for k in kernels}.get(dom["index"], "")
    peak = stage_peak_tflops(kern, dom["name"], prec)
    if kern:
        achieved = dom["flops"] / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    elif peak:
        # FP64 eigensolvers: vector-ALU and LDS-latency bound work priced at the FP64 rate
        achieved = dom["flops"] / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    else:
        achieved = dom["bytes"] / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom["name"], cfg, prec)
    roof["kernel"] = dom["name"]
    roof["avg_launch_ms"] = avg_ms
    roof["launches_timed"] = dstage["launches"]
    e2e, gemm_phase = roofline_fractions(prof, kernels, prec, sec * 1e3)

    out = {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[cfg], "precision": prec, "instances": len(wl.instances),
                   "electrons": wl.n_electrons, "gradient": args.gradient, "expm": args.expm,
                   "odd_lambda": args.odd_lambda, "overlap": args.overlap},
        "create_ms": t_create * 1e3,
        "tflops": total_flops / sec / 1e12,
        "ms_per_step_eager": sec_eager * 1e3,
        "roofline": roof,
        "roofline_end_to_end": e2e,
        "roofline_gemm_phase": gemm_phase,
        "parity": {"max_dE_per_electron": dE, "max_rel_dg": dg, "max_elementwise_dg": de,
                   "target_dE_per_electron": 1e-8, "target_rel_dg": 1e-6, "oracle": route},
        "stages_ms": {r["name"]: round(r["total_ms"] / max(r["launches"], 1), 5) for r in prof if r["launches"]},
        "gemm_kernels": gemm_kernel_table(h, prof),
    }
    if not args.no_fp64_compare and prec != "fp64":
        log("FP64 path")
        h64, A64, E64, G64 = build_handle(wl, "fp64", args.gemm_tuning, args.gradient, args.expm, args.odd_lambda)
        h64.set_graph(True)
        sec64, _ = timed_run(h64, A64, E64, G64, max(5, args.steps // 2), 2)
        out["fp64_path"] = {"value": 1.0 / sec64, "ms_per_step": sec64 * 1e3, "speedup": sec64 / sec}
        h64.close()
        del A64, E64, G64
    if lbfgs_iters > 0:
        log("L-BFGS iterations")
        # full L-BFGS iterations from A = 0 (direction, line search, memory update)
        from paper_2101_12597_amd import lbfgs_defaults
        lp = lbfgs_defaults()
        lp.reset_norm = args.lbfgs_reset_norm
        h.set_graph(True)
        A0 = torch.zeros_like(A)
        info = h.lbfgs_step(A0, E, G, lp)  # initialisation + first iteration
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [h.lbfgs_step(A0, E, G, lp) for _ in range(lbfgs_iters)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / lbfgs_iters
        out["lbfgs"] = {"ms_per_iteration": dt * 1e3, "iterations": lbfgs_iters,
                        "evals_per_iteration": (infos[-1]["n_evals"] - info["n_evals"]) / lbfgs_iters,
                        "E": infos[-1]["E"], "gnorm": infos[-1]["gnorm"],
                        "reset_norm": args.lbfgs_reset_norm,
                        "resets": sum(1 for i in infos if i["flags"] & 1)}
        h.set_graph(False)
    if not args.no_cpu_baseline:
        # the oracle as timed above, repeated (at most 8 times) until about 10 s of work
        reps, total = 1, t_oracle
        with blas_limit(args.cpu_threads):
            while total < 10.0 and reps < 8:
                total += oracle_reference(wl, params, args.gradient, args.expm, args.odd_lambda)[2]
                reps += 1
        out["cpu_baseline"] = {
            "value": reps / total, "unit": "evals/s", "cores": oracle_threads, "kind": "oracle",
            "sample": f"{reps} full evaluation(s) of all {len(wl.instances)} instances with the FP64 "
                      f"oracle's {route} ({args.gradient} gradient), NumPy/OpenBLAS with "
                      f"{oracle_threads} threads",
            "cpu_model": cpu_model(), "threads": oracle_threads,
        }
    h.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
