"""Batched refactorization benchmark: many matrices of uneven size.

Workload: 64 independent circuit matrices from the generator without rails,
n drawn log-uniform in [1,000, 50,000] (seeds 3000 + i), each refactorized
with new values (every nonzero times a log-normal(0, 0.1) factor) and solved
for 4 right-hand sides uniform in [-1, 1].  Three ways are timed on the
device-resident values:
  * plain FP64 per matrix: glu_refactor + glu_solve, one matrix after another;
  * batched FP64: one glu_batch_factor (shared level wavefronts from a
    captured graph) + one glu_batch_solve (every solve at once);
  * batched mixed form: FP32 sparse levels (precision = 1) in one
    glu_batch_factor, then one glu_batch_solve refining every handle in FP64
    to backward error <= 1e-13.
All computation is in the HIP library; this module chooses arguments and
times.  Prints one JSON line.

    python -m paper_1908_00204_amd.batch_bench [--count 64] [--rounds 3]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import glu


def main() -> int:
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import scipy.sparse as sp
    import torch

    import circuitgen as cg

    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--rounds", type=int, default=3)
    ap.add_argument("--nrhs", type=int, default=4)
    args = ap.parse_args()
    rng = np.random.default_rng(3000)
    mats = []
    for i in range(args.count):
        n = int(round(np.exp(rng.uniform(np.log(1000), np.log(50000)))))
        mats.append(cg.circuit_matrix(n, seed=3000 + i))
    dev = torch.device("cuda:0")
    rhs = [torch.from_numpy(np.ascontiguousarray(cg.rhs(A.n, args.nrhs, 3500 + i).T)).to(dev).t()
           for i, A in enumerate(mats)]
    vals = [[torch.from_numpy(cg.perturbed_values(A.values, 3000 + 10**6 + 100 * r + i)).to(dev)
             for i, A in enumerate(mats)] for r in range(args.rounds)]
    stream = torch.cuda.current_stream()

    def handles(precision):
        hs = []
        for A in mats:
            h = glu.Handle(device=0, precision=precision)
            h.analyze(A.n, A.colptr, A.rowind)
            hs.append(h)
        return hs

    def berr_max(hs, xs, r):
        worst = 0.0
        for A, x, b, v in zip(mats, xs, rhs, vals[r]):
            M = sp.csc_matrix((v.cpu().numpy(), A.rowind, A.colptr), shape=(A.n, A.n))
            normA = abs(M).sum(axis=1).max()
            xh, bh = x.cpu().numpy(), b.cpu().numpy()
            for c in range(xh.shape[1]):
                worst = max(worst, np.abs(M @ xh[:, c] - bh[:, c]).max() / (normA * np.abs(xh[:, c]).max()))
        return float(worst)

    def run(kind):
        hs = handles(1 if kind == "batched_mixed" else 0)
        batch = glu.Batch(hs) if kind != "per_matrix_fp64" else None
        xs = [torch.empty((args.nrhs, A.n), dtype=torch.float64, device=dev).t() for A in mats]
        times, iters, split = [], [], []
        for r in range(args.rounds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if batch is None:
                for h, v, b, x in zip(hs, vals[r], rhs, xs):
                    h.factor(v, stream=stream)
                    h.solve(b, x, stream=stream)
            else:
                batch.factor(vals[r], stream=stream)
                batch.solve(rhs, xs, stream=stream)
                iters.extend(h.query()["refine_iters"] for h in hs)
                q = batch.query()
                split.append((q["t_levels_ms"], q["t_total_ms"], q["t_solve_ms"]))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = float(np.median(times[1:] if len(times) > 1 else times))
        out = {"seconds_per_round": t, "solves_per_s": args.count * args.nrhs / t,
               "backward_error_max": berr_max(hs, xs, args.rounds - 1)}
        if batch is not None:
            lv, fa, so = (float(np.median([x[k] for x in split])) for k in range(3))
            out.update({"wavefronts": batch.query()["n_wavefronts"], "captured": batch.query()["captured"],
                        "factor_ms": fa, "factor_levels_ms": lv, "solve_ms": so})
            batch.close()
        if kind == "batched_mixed":
            out["refine_iters_mean"] = float(np.mean(iters))
            out["fp64_fallbacks"] = int(sum(h.query()["fp64_fallback"] for h in hs))
        for h in hs:
            h.close()
        print(f"[batch] {kind}: {out}", file=sys.stderr, flush=True)
        return out

    res = {k: run(k) for k in ("per_matrix_fp64", "batched_fp64", "batched_mixed")}
    base = res["per_matrix_fp64"]["solves_per_s"]
    print(json.dumps({"metric": "solves/s, 64 matrices of n log-uniform in [1e3, 5e4], 4 RHS each",
                      "count": args.count, "n": [A.n for A in mats], **res,
                      "speedup_batched_fp64": res["batched_fp64"]["solves_per_s"] / base,
                      "speedup_batched_mixed": res["batched_mixed"]["solves_per_s"] / base}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
