#!/usr/bin/env python3
"""Benchmark of the levelized sparse LU path on one MI355X.

A step is one pass of the numeric hot path over the benchmark matrix: refactor
with the step's values (value load, the level-by-level normalisation and
submatrix update, pivot check) followed by one forward/backward solve.  The
pattern is analyzed once before timing (ordering, symbolic fill, relaxed DAG,
levels, plan: reported separately), as in a Newton loop.  Inputs are resident
in device memory when the timed region starts.

Workload (default): circuit-like matrix n=100,000 with 150 supply rails each
wired to 2% of the nodes, one right-hand side uniform in [-1, 1].

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "refactor ms & solves/s at backward error ≤1e-12; p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6

WORKLOADS = {
    "c0": "circuit n=2,000 (no rails), refactor + 1 solve",
    "c1": "circuit n=100,000 with 150 rails at 2% connectivity, refactor + 1 solve",
}


def kernel_source_sha() -> str:
    p = os.path.join(ROOT, "paper_1908_00204_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def work_model(sym: dict, tail_m: int, schur_macs: int) -> dict:
    """Algorithmic work of one factorization, split at the dense block.

    Sparse levels (columns j < t = n - tail_m, every product whose target is
    outside the dense block), right-looking scatter model: 8 B per column
    (pivot), 20 B per L entry (read index and value, write the normalised
    value), 16 B per U entry (value and target position) and 20 B per
    multiply-add (target read + write, row index).
    Schur-complement update of the block from the columns before it: the
    nonzero products sum_j |L(t:n,j)| |U(j,t:n)|.
    Dense block of order m: 2/3 m^3 + O(m^2) flops of a no-pivot LU."""
    n = len(sym["lu_colptr"]) - 1
    cp, ri = sym["lu_colptr"], sym["lu_rowind"]
    cols = np.repeat(np.arange(n), np.diff(cp))
    nl = np.bincount(cols[ri > cols], minlength=n).astype(np.int64)
    nu = np.bincount(ri[ri < cols], minlength=n).astype(np.int64)
    t = n - tail_m
    macs = int((nl[:t] * nu[:t]).sum()) - schur_macs
    sparse_bytes = 8 * t + 20 * int(nl[:t].sum()) + 16 * int(nu[:t].sum()) + 20 * macs
    m = tail_m
    dense_flops = sum((m - k - 1) + 2 * (m - k - 1) ** 2 for k in range(m))
    return {"sparse_macs": macs, "sparse_bytes": sparse_bytes, "dense_flops": dense_flops,
            "schur_macs": schur_macs}


def stored_traffic(config: str):
    """HBM traffic of the level loop from committed rocprofv3 counter runs, only
    if they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"k_level_traffic_{config}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_src_sha") != kernel_source_sha():
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


def cpu_baseline(A, sym: dict, b: np.ndarray) -> dict:
    """The oracle (single-threaded C, Gilbert-Peierls left-looking) on the same
    matrix: one numeric factorization + one solve, its symbolic pattern computed
    beforehand and not timed."""
    import oracle

    B = oracle.permute(A, sym["perm"])
    t0 = time.perf_counter()
    val = oracle.factor(B, sym["lu_colptr"], sym["lu_rowind"])
    t1 = time.perf_counter()
    oracle.solve(sym["lu_colptr"], sym["lu_rowind"], val, sym["perm"], b)
    t2 = time.perf_counter()
    return {
        "value": 1.0 / (t2 - t0),
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one factor ({(t1 - t0):.2f} s) + one solve ({(t2 - t1) * 1e3:.1f} ms) of the same "
                  f"n={A.n} matrix on one host core; symbolic analysis excluded",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    A = cg.config_matrix(args.config)
    b_host = cg.rhs(A.n, 1, seed=1000 * int(args.config[1:]) + 500)
    print(f"[bench] {args.config}: n={A.n} nnz={A.nnz}; analyzing", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    h = glu.Handle(device=0)
    h.analyze(A.n, A.colptr, A.rowind)
    t_analyze = (time.perf_counter() - t0) * 1e3
    q = h.query()
    print(f"[bench] analyzed in {t_analyze:.0f} ms: nnz_lu={q['nnz_lu']} levels={q['n_levels']} "
          f"macs={q['macs']:.3e}", file=sys.stderr, flush=True)

    base = torch.from_numpy(A.values).to(dev)
    steps_vals = []
    for r in range(args.warmup + args.steps):
        v = cg.perturbed_values(A.values, seed=1000 * int(args.config[1:]) + 10**6 + r)
        steps_vals.append(torch.from_numpy(v).to(dev))
    bd = torch.from_numpy(b_host[:, 0].copy()).to(dev)
    xd = torch.empty_like(bd)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    for r in range(args.warmup):
        h.refactor(steps_vals[r], stream=stream) if r else h.factor(steps_vals[r], stream=stream)
        h.solve(bd, xd, stream=stream)
    if args.warmup == 0:
        h.factor(base, stream=stream)
    torch.cuda.synchronize()
    print("[bench] warm-up done; timing", file=sys.stderr, flush=True)

    upd_ms, fac_ms, sol_ms, dense_ms, schur_ms = [], [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(args.steps):
        h.refactor(steps_vals[args.warmup + r], stream=stream)
        qq = h.query()
        upd_ms.append(qq["t_update_ms"])
        dense_ms.append(qq["t_dense_ms"])
        schur_ms.append(qq["t_schur_ms"])
        fac_ms.append(qq["t_factor_ms"])
        h.solve(bd, xd, stream=stream)
        sol_ms.append(h.query()["t_solve_ms"])
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
    Al = cg.CscMatrix(A.n, A.colptr, A.rowind, last_vals)
    x = xd.cpu().numpy()
    be = backward_error(Al, x, b_host[:, 0])

    sym = h.export_symbolic()
    wm = work_model(sym, q["tail_m"], q["schur_macs"])
    upd = float(np.mean(upd_ms))
    dns = float(np.mean(dense_ms))
    achieved = wm["sparse_bytes"] / (upd * 1e-3) / 1e9
    tr = stored_traffic(args.config)
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
    sch = float(np.mean(schur_ms))
    dns = dns - sch  # dense LU + scatter + pivot check
    dense_tf = wm["dense_flops"] / (dns * 1e-3) / 1e12 if dns > 0 else 0.0
    sch_exec = 2 * 256 * q["schur_steps"]  # FMAs the 16 x 16 tile steps execute, as flops
    roofline_schur = {
        "bound": "alu",
        "kernel": "Schur-complement update of the dense block (gather, panels, 16x16 tiles, FP64 FMA)",
        "achieved": sch_exec / (sch * 1e-3) / 1e12 if sch > 0 else 0.0,
        "peak": FP64_PEAK_TFS,
        "unit": "TFLOP/s",
        "frac": (sch_exec / (sch * 1e-3) / 1e12 / FP64_PEAK_TFS) if sch > 0 else 0.0,
        "useful_flops": 2 * wm["schur_macs"],
        "executed_flops": sch_exec,
        "launch_ms": sch,
    }
    roofline_dense = {
        "bound": "mfma",
        "kernel": "dense trailing block (gather, blocked LU with FP64 MFMA update, scatter)",
        "achieved": dense_tf,
        "peak": FP64_PEAK_TFS,
        "unit": "TFLOP/s",
        "frac": dense_tf / FP64_PEAK_TFS,
        "traffic": None,
        "flops": wm["dense_flops"],
        "launch_ms": dns,
        "m": q["tail_m"],
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
        "dtype": "f64",
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
        "refactor_split_ms": {"levels": upd, "schur": sch, "dense_lu": dns},
        "solve_ms": float(np.median(sol_ms)),
        "backward_error": be,
        "analyze_ms": {"total": t_analyze, "order": q["t_order_ms"], "symbolic": q["t_symbolic_ms"],
                       "dag_levels": q["t_levels_ms"], "plan_upload": q["t_plan_ms"]},
        "roofline": roofline,
        "roofline_dense": roofline_dense,
        "roofline_schur": roofline_schur,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle, one core)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(A, sym, b_host[:, 0])
    h.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
