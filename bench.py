#!/usr/bin/env python3
"""Benchmark of the levelized sparse LU path on one MI355X.

A step is one pass of the numeric hot path over the benchmark matrix: refactor
with the step's values (value load, the level-by-level normalisation and
submatrix update, the dense trailing block, pivot check) followed by one
forward/backward solve.  The pattern is analyzed once before timing
(ordering, symbolic fill, relaxed DAG, levels, plan: reported separately), as
in a Newton loop whose values change every round.  Inputs are resident in
device memory when the timed region starts.

Workloads (``--config``):
  c2 (default): circuit-like matrix n=1,000,000 with 400 supply rails each
      wired to 0.5% of the nodes; every step refactors with every nonzero
      scaled by an independent log-normal(0, 0.1) factor (relative to the
      base values) and solves one right-hand side uniform in [-1, 1].
  c1: n=100,000 with 150 rails at 2%, same step.
  c0: n=2,000 without rails (the latency case), same step.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "refactor ms & solves/s at backward error ≤1e-12; p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3   # dense FP32 matrix-core peak
FP32_BLOCK_MIN = 8192   # the mixed form factorizes dense blocks of at least this many (padded) columns in FP32

WORKLOADS = {
    "c0": "circuit n=2,000 (no rails), refactor + 1 solve per step",
    "c1": "circuit n=100,000 with 150 rails at 2% connectivity, refactor + 1 solve per step",
    "c2": "circuit n=1,000,000 with 400 rails at 0.5% connectivity, Newton-like refactor "
          "(log-normal(0,0.1) value changes, fixed pattern) + 1 solve per step",
}


def kernel_source_sha(src: str = "kernels.hip") -> str:
    p = os.path.join(ROOT, "paper_1908_00204_amd", "csrc", src)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def work_model(q: dict, vbytes: int = 8) -> dict:
    """Algorithmic work of one factorization, split at the dense block, from
    the analysis counts.

    Sparse levels (columns j < t = n - m, every product whose target is outside
    the dense block), right-looking scatter model with values of vbytes bytes
    (8 in FP64, 4 in the mixed form's FP32 levels): one value per column
    (pivot), per L entry a 4 B index and a value read and written (20 B in
    FP64), per U entry its value and an 8 B target position (16 B), per
    multiply-add the target read and written and a 4 B row index (20 B).  Schur-complement update of the block from the
    columns before it: its nonzero products.  Dense block of order m: the
    method's own products inside it (tail_macs) and, beside them, the flops a
    dense no-pivot LU of order m executes (2/3 m^3 + O(m^2))."""
    m = q["tail_m"]
    t = q["n"] - m
    sparse_bytes = (vbytes * t + (4 + 2 * vbytes) * q["level_nl"] + (8 + vbytes) * q["level_nu"]
                    + (4 + 2 * vbytes) * q["level_macs"])
    dense_exec = sum((m - k - 1) + 2 * (m - k - 1) ** 2 for k in range(m))
    return {"sparse_macs": q["level_macs"], "sparse_bytes": sparse_bytes,
            "tail_method_flops": 2 * q["tail_macs"] + (m * (m - 1)) // 2 if m else 0,
            "dense_exec_flops": dense_exec, "schur_macs": q["schur_macs"]}


def stored_traffic(config: str, tail_m: int, family: str = "k_level", src: str = "kernels.hip"):
    """HBM traffic of a kernel family from committed rocprofv3 counter runs,
    only if they were taken on the current kernel source and the same plan
    (the same dense block size)."""
    p = os.path.join(ROOT, "profiles", f"{family}_traffic_{config}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_src_sha") != kernel_source_sha(src) or d.get("dense_tail") != tail_m:
        return None
    return d


def backward_error(A, x, b) -> float:
    import scipy.sparse as sp

    M = sp.csc_matrix((A.values, A.rowind, A.colptr), shape=(A.n, A.n))
    normA = abs(M).sum(axis=1).max()
    x = x.reshape(A.n, -1)
    b = b.reshape(A.n, -1)
    return max(float(np.abs(M @ x[:, c] - b[:, c]).max() / (normA * np.abs(x[:, c]).max()))
               for c in range(x.shape[1]))


def host_cpu() -> dict:
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_available": avail}


def cpu_baseline(config: str, A, q: dict, perm: np.ndarray | None) -> dict:
    """The oracle (single-threaded C, Gilbert-Peierls left-looking) on one
    host core: one numeric factorization + one solve; the oracle's own
    symbolic step on the same ordering runs beforehand and is not timed.
    c0/c1 run on the workload's own matrix (c0 repeated for at least 2 s);
    c2 (about 8e12 multiply-adds, hours on one core) runs the n=100,000
    matrix of the same generator and is scaled by the multiply-add counts."""
    import circuitgen as cg
    import oracle

    scaled = config == "c2"
    if scaled:
        from paper_1908_00204_amd import glu

        A = cg.config_matrix("c1")
        hp = glu.Handle(device=-1)  # host-only: the same ordering as the GPU path, as data
        perm = hp.analyze(A.n, A.colptr, A.rowind).export_symbolic()["perm"]
        hp.close()
    r = oracle.analyze(A, perm, numeric=False)
    B, lcp, lri = r.B, r.lu_colptr, r.lu_rowind
    st = oracle.level_stats(A.n, lcp, lri, r.level_ptr, r.level_cols)
    b = cg.rhs(A.n, 1, 7)[:, 0]
    reps, t_fac, t_sol = 0, 0.0, 0.0
    while reps == 0 or (t_fac + t_sol < 2.0 and reps < 1000):
        t0 = time.perf_counter()
        val = oracle.factor(B, lcp, lri)
        t1 = time.perf_counter()
        oracle.solve(lcp, lri, val, r.perm, b)
        t2 = time.perf_counter()
        t_fac += t1 - t0
        t_sol += t2 - t1
        reps += 1
    t_fac /= reps
    t_sol /= reps
    cpu = host_cpu()
    out = {"cores": 1, "kind": "oracle", "unit": "solves/s", "host_cpu": cpu}
    if not scaled:
        out["value"] = 1.0 / (t_fac + t_sol)
        out["sample"] = (f"{reps} x (one factor {t_fac:.3f} s + one solve {t_sol * 1e3:.2f} ms) of the same "
                         f"n={A.n} matrix on one host core; symbolic analysis excluded")
    else:
        mac_rate = st["macs"] / t_fac
        nnz_rate = (st["nL"] + st["nU"] + A.n) / t_sol
        est = q["macs"] / mac_rate + q["nnz_lu"] / nnz_rate
        out["value"] = 1.0 / est
        out["sample"] = (f"oracle measured on the n=100,000 matrix of the same generator (AMD order): "
                         f"factor {t_fac:.2f} s for {st['macs']:.3e} multiply-adds ({mac_rate / 1e9:.2f} GMAC/s), "
                         f"solve {t_sol * 1e3:.1f} ms; scaled to the n=1,000,000 pattern ({q['macs']:.3e} "
                         f"multiply-adds, {q['nnz_lu']:.3e} factor entries): {est:.0f} s per factor + solve")
    return out


def machine_probes(dev) -> dict:
    """Achievable references on this GPU: a plain device copy (HBM read +
    write) and a large FP64 GEMM (matrix cores, library kernel)."""
    import torch

    nb = 1 << 31
    src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    best = 1e9
    for _ in range(5):
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    copy_gbs = 2 * nb / (best * 1e-3) / 1e9
    del src, dst
    n = 8192
    a = torch.rand(n, n, dtype=torch.float64, device=dev)
    bm = torch.rand(n, n, dtype=torch.float64, device=dev)
    c = a @ bm
    best = 1e9
    for _ in range(3):
        e0.record()
        c = a @ bm
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    gemm_tfs = 2 * n ** 3 / (best * 1e-3) / 1e12
    del a, bm, c
    torch.cuda.empty_cache()
    return {"hbm_copy_GBs": copy_gbs, "hbm_copy_bytes": 2 * nb, "fp64_gemm_TFs": gemm_tfs,
            "fp64_gemm_n": n, "hbm_peak_GBs": HBM_PEAK_GBS, "fp64_peak_TFs": FP64_PEAK_TFS}


def pct(v, p):
    return float(np.percentile(np.asarray(v), p))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dense-tail", type=int, default=0,
                    help="dense trailing block: 0 = cost model, -1 = none, m > 0 = the last m columns")
    ap.add_argument("--precision", type=int, default=0, choices=(0, 1),
                    help="0 = plain FP64 (the reported workload); 1 = the mixed form (FP32 factors, FP64 refinement)")
    ap.add_argument("--dense-gemm", type=int, default=0, choices=(0, 1),
                    help="dense block bulk updates: 0 = BLAS library DGEMM, 1 = own MFMA kernel")
    ap.add_argument("--no-probes", action="store_true", help="skip the copy / GEMM reference probes")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB on the device once "
                         "(a plain copy of known size that calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path runs on a single MI355X)", file=sys.stderr)
        return 2

    import torch

    import circuitgen as cg
    from paper_1908_00204_amd import glu

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    cfg = int(args.config[1:])
    A = cg.config_matrix(args.config)
    b_host = cg.rhs(A.n, 1, seed=1000 * cfg + 500)
    print(f"[bench] {args.config}: n={A.n} nnz={A.nnz}; analyzing", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    h = glu.Handle(device=0, dense_gemm=args.dense_gemm, dense_tail=args.dense_tail, precision=args.precision)
    h.analyze(A.n, A.colptr, A.rowind)
    t_analyze = (time.perf_counter() - t0) * 1e3
    import resource

    peak_host_gb = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss * 1024 / 1e9  # ru_maxrss is KiB on Linux
    q = h.query()
    print(f"[bench] analyzed in {t_analyze:.0f} ms: nnz_lu={q['nnz_lu']} levels={q['n_levels']} "
          f"macs={q['macs']:.3e} tail={q['tail_m']}", file=sys.stderr, flush=True)

    nval = args.warmup + args.steps
    steps_vals = []
    for r in range(nval):
        v = cg.perturbed_values(A.values, seed=1000 * cfg + 10**6 + r)
        steps_vals.append(torch.from_numpy(v).to(dev))
    bd = torch.from_numpy(b_host[:, 0].copy()).to(dev)
    xd = torch.empty_like(bd)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    t_first = time.perf_counter()
    h.factor(steps_vals[0], stream=stream)
    h.solve(bd, xd, stream=stream)
    first_ms = (time.perf_counter() - t_first) * 1e3
    for r in range(1, args.warmup):
        h.refactor(steps_vals[r], stream=stream)
        h.solve(bd, xd, stream=stream)
    torch.cuda.synchronize()
    print(f"[bench] first factor+solve {first_ms:.1f} ms; warm-up done; timing", file=sys.stderr, flush=True)

    upd_ms, fac_ms, sol_ms, dense_ms, schur_ms, step_ms, refine_iters = [], [], [], [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(args.steps):
        ts = time.perf_counter()
        h.refactor(steps_vals[args.warmup + r], stream=stream)
        h.solve(bd, xd, stream=stream)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        # the device-event times of this step's factorization and solve, read
        # after the step (inside the timed loop, so ms_per_step includes them)
        qq = h.query()
        upd_ms.append(qq["t_update_ms"])
        dense_ms.append(qq["t_dense_ms"])
        schur_ms.append(qq["t_schur_ms"])
        fac_ms.append(qq["t_factor_ms"])
        refine_iters.append(qq["refine_iters"])
        sol_ms.append(qq["t_solve_ms"])
        if args.steps >= 10 and (r + 1) % max(1, args.steps // 5) == 0:
            print(f"[bench] step {r + 1}/{args.steps}: {step_ms[-1]:.2f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # accuracy of the last step
    last_vals = steps_vals[-1].cpu().numpy()
    del steps_vals
    Al = cg.CscMatrix(A.n, A.colptr, A.rowind, last_vals)
    x = xd.cpu().numpy()
    be = backward_error(Al, x, b_host[:, 0])

    probes = None
    if not args.no_probes:
        print("[bench] reference probes (device copy, FP64 GEMM)", file=sys.stderr, flush=True)
        probes = machine_probes(dev)

    wm = work_model(q, 8 if args.precision == 0 else 4)
    # the mixed form factorizes large dense blocks in FP32 (the FP32 matrix-core peak applies)
    fp32_block = (args.precision == 1 and args.dense_gemm == 0 and q["tail_m"] > 0
                  and (q["tail_m"] + 63) // 64 * 64 >= FP32_BLOCK_MIN)
    dense_peak = FP32_PEAK_TFS if fp32_block else FP64_PEAK_TFS
    upd = float(np.mean(upd_ms))
    sch = float(np.mean(schur_ms))
    dns = float(np.mean(dense_ms)) - sch  # dense LU + pivot check
    fac = float(np.mean(fac_ms))
    achieved = wm["sparse_bytes"] / (upd * 1e-3) / 1e9 if upd > 0 else 0.0
    # (the stored level traffic was counted on the FP64 level kernels)
    tr = stored_traffic(args.config, q["tail_m"]) if args.precision == 0 else None
    roofline = {
        "bound": "hbm",
        "kernel": "k_level (per-level normalisation + submatrix update launches, sparse levels)",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": None if tr is None else tr["bytes_per_factorization"],
        "algorithmic_bytes": wm["sparse_bytes"],
        "launch_ms": upd,
    }
    if probes:
        roofline["frac_of_measured_copy"] = achieved / probes["hbm_copy_GBs"]
    useful_sch = 2 * wm["schur_macs"]
    sch_exec = 2 * 256 * q["schur_steps"]  # FMAs the 16 x 16 tile steps execute, as flops
    roofline_schur = {
        "bound": "mfma",
        "kernel": "Schur-complement update of the dense block (gather, panels, 16x16 FP64 MFMA tiles)",
        "achieved": useful_sch / (sch * 1e-3) / 1e12 if sch > 0 else 0.0,
        "peak": FP64_PEAK_TFS,
        "unit": "TFLOP/s",
        "frac": (useful_sch / (sch * 1e-3) / 1e12 / FP64_PEAK_TFS) if sch > 0 else 0.0,
        "basis": "useful flops (2 x nonzero products)",
        "useful_flops": useful_sch,
        "executed_flops": sch_exec,
        "executed_frac": (sch_exec / (sch * 1e-3) / 1e12 / FP64_PEAK_TFS) if sch > 0 else 0.0,
        "launch_ms": sch,
    }
    meth = wm["tail_method_flops"]
    roofline_dense = {
        "bound": "mfma",
        "kernel": ("dense trailing block (FP32 copy, ROCm LAPACK no-pivot LU, widened back; pivot check)"
                   if fp32_block else
                   "dense trailing block (blocked no-pivot LU: FP64 MFMA panel kernels, bulk updates through "
                   "the ROCm BLAS DGEMM; pivot check)" if args.dense_gemm == 0 else
                   "dense trailing block (blocked no-pivot LU, every update on this library's FP64 MFMA kernels; "
                   "pivot check)"),
        "achieved": meth / (dns * 1e-3) / 1e12 if dns > 0 else 0.0,
        "peak": dense_peak,
        "unit": "TFLOP/s",
        "frac": (meth / (dns * 1e-3) / 1e12 / dense_peak) if dns > 0 else 0.0,
        "basis": "the method's own flops inside the block (2 x products + divisions)",
        "method_flops": meth,
        "dense_equivalent_flops": wm["dense_exec_flops"],
        "dense_equivalent_frac": (wm["dense_exec_flops"] / (dns * 1e-3) / 1e12 / dense_peak) if dns > 0 else 0.0,
        "launch_ms": dns,
        "m": q["tail_m"],
    }
    # combined roofline of the refactorization: sparse levels at HBM speed,
    # the block's products (Schur update + LU, the method's own flops) at the
    # matrix-core peak of their precision
    t_roof = (wm["sparse_bytes"] / (HBM_PEAK_GBS * 1e9) + useful_sch / (FP64_PEAK_TFS * 1e12)
              + meth / (dense_peak * 1e12))
    roofline_refactor = {
        "model": ("sparse-level algorithmic bytes / 8 TB/s + Schur method flops / 78.6 TFLOP/s + dense-block "
                  f"method flops / {dense_peak} TFLOP/s"),
        "t_roof_ms": t_roof * 1e3,
        "t_measured_ms": fac,
        "frac": t_roof * 1e3 / fac if fac > 0 else 0.0,
    }
    out = {
        "metric": METRIC,
        "value": 1e3 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32 factors + f64 refinement",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.config],
            "n": A.n,
            "nnz_a": int(A.nnz),
            "nnz_lu": q["nnz_lu"],
            "macs": q["macs"],
            "levels": q["n_levels"],
            "levels_launched": q["n_exec_levels"],
            "levels_per_mode": q["n_levels_mode"],
            "dense_tail": q["tail_m"],
            "ordering": "amd",
            "nrhs": 1,
        },
        "refactor_ms": float(np.median(fac_ms)),
        "refactor_ms_p10_p90": [pct(fac_ms, 10), pct(fac_ms, 90)],
        "step_ms_p10_p50_p90": [pct(step_ms, 10), pct(step_ms, 50), pct(step_ms, 90)],
        "refactor_split_ms": {"levels": upd, "schur": sch, "dense_lu": dns},
        "solve_ms": float(np.median(sol_ms)),
        "first_factor_solve_ms": first_ms,
        "backward_error": be,
        "refine_iters_mean": float(np.mean(refine_iters)) if args.precision == 1 else None,
        "analyze_peak_host_gb": peak_host_gb,
        "analyze_ms": {"total": t_analyze, "order": q["t_order_ms"], "symbolic": q["t_symbolic_ms"],
                       "dag_levels": q["t_levels_ms"], "plan_upload": q["t_plan_ms"]},
        "device_bytes": q["device_bytes"],
        "dense_bulk_update": "BLAS library DGEMM" if args.dense_gemm == 0 else "own FP64 MFMA kernel",
        "roofline": None,
        "roofline_levels": roofline,
        "roofline_dense": roofline_dense,
        "roofline_schur": roofline_schur,
        "roofline_refactor": roofline_refactor,
        "machine": probes,
        "cpu_baseline": None,
    }
    # the roofline of the dominant kernel family (most device time per step)
    # (the stored dense traffic was counted on the FP64 block LU)
    dtr = None if fp32_block else stored_traffic(args.config, q["tail_m"], "dense", "dense_tail.hip")
    roofline_dense["traffic"] = None if dtr is None else dtr["bytes_per_factorization"]
    fam = max((upd, "levels"), (sch, "schur"), (dns, "dense"))[1]
    dom = {"levels": roofline, "schur": roofline_schur, "dense": roofline_dense}[fam]
    out["roofline"] = dict(dom, family=fam)
    if "traffic" not in out["roofline"]:
        out["roofline"]["traffic"] = None
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle, one core)", file=sys.stderr, flush=True)
        perm = h.export_symbolic()["perm"] if args.config != "c2" else None
        out["cpu_baseline"] = cpu_baseline(args.config, A, q, perm)
    h.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
