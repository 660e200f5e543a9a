"""Threshold autotuner and mode ablation for the level kernels.

The paper chooses its stream-mode threshold by a sweep (Section IV, the
threshold figure) and measures what each kernel mode is worth by switching it
off (Table 3).  This module does both on MI355X through the C ABI: it times
the numeric refactorization of one pattern under different plan settings
(level-width thresholds of the three modes, the dense trailing block) and
returns the fastest; every setting gives the same factors up to rounding
order, so tuning never changes what is computed.  Everything runs in the HIP
library; this module only chooses arguments and reads timings.

Usage:
    python -m paper_1908_00204_amd.autotune --config c1 [--ablation] [--steps 10]
prints one JSON object (the timings of every setting and the chosen one).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import glu


def time_setting(A, values, steps: int = 10, **kw) -> dict:
    """Analyze A under the Handle keyword settings kw, factor once, then time
    `steps` refactorizations with the given value arrays (device tensors,
    used round robin) and one solve; medians of the device times (HIP events
    inside the library)."""
    import torch

    h = glu.Handle(device=0, **kw)
    t0 = time.perf_counter()
    h.analyze(A.n, A.colptr, A.rowind)
    t_an = (time.perf_counter() - t0) * 1e3
    stream = torch.cuda.current_stream()
    h.factor(values[0], stream=stream)
    b = torch.ones(A.n, dtype=torch.float64, device=values[0].device)
    x = torch.empty_like(b)
    fac, lev, sol = [], [], []
    for r in range(steps):
        h.refactor(values[(r + 1) % len(values)], stream=stream)
        q = h.query()
        fac.append(q["t_factor_ms"])
        lev.append(q["t_update_ms"])
        h.solve(b, x, stream=stream)
        sol.append(h.query()["t_solve_ms"])
    q = h.query()
    h.close()
    return {"settings": kw, "refactor_ms": float(np.median(fac)), "levels_ms": float(np.median(lev)),
            "solve_ms": float(np.median(sol)), "analyze_ms": t_an, "levels_launched": q["n_exec_levels"],
            "levels_per_mode": q["n_levels_mode"], "tail_m": q["tail_m"]}


def ablation_settings() -> list[dict]:
    """The Table 3 analogue: the automatic plan, then each mode switched off
    (its levels fall to the neighbouring mode), then each mode on every level,
    with and without the dense trailing block."""
    out = []
    for tail in (0, -1):
        base = {"dense_tail": tail}
        out += [
            dict(base),                                                       # automatic plan
            dict(base, stream_threshold=-1),                                  # no stream mode
            dict(base, large_threshold=-1),                                   # no large-block mode
            dict(base, force_mode=glu.GLU_MODE_SMALL_BLOCK),                  # small-block everywhere
            dict(base, force_mode=glu.GLU_MODE_LARGE_BLOCK),                  # large-block everywhere
            dict(base, force_mode=glu.GLU_MODE_STREAM),                       # stream mode everywhere
        ]
    return out


def threshold_settings() -> list[dict]:
    """The threshold sweep: stream-mode width threshold x large-block width
    threshold, with the cost model's dense block."""
    out = []
    for st in (1, 4, 16, 64, 256):
        for lt in (-1, 512, 4096):
            if lt != -1 and lt <= st:
                continue
            out.append({"stream_threshold": st, "large_threshold": lt})
    return out


def tune(A, values, steps: int = 5, settings: list[dict] | None = None) -> dict:
    """Time every setting; return {"results": [...], "best": settings}."""
    res = [time_setting(A, values, steps, **s) for s in (settings or threshold_settings())]
    best = min(res, key=lambda r: r["refactor_ms"])
    return {"results": res, "best": best["settings"]}


def main() -> int:
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import circuitgen as cg

    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c1", choices=["c0", "c1"])
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--ablation", action="store_true", help="mode ablation instead of the threshold sweep")
    args = ap.parse_args()
    A = cg.config_matrix(args.config)
    cfg = int(args.config[1:])
    vals = [torch.from_numpy(cg.perturbed_values(A.values, seed=1000 * cfg + 10**6 + r)).cuda() for r in range(4)]
    settings = ablation_settings() if args.ablation else threshold_settings()
    res = []
    for s in settings:
        r = time_setting(A, vals, args.steps, **s)
        print(f"[autotune] {args.config} {s}: refactor {r['refactor_ms']:.3f} ms (levels {r['levels_ms']:.3f}), "
              f"solve {r['solve_ms']:.3f} ms", file=sys.stderr, flush=True)
        res.append(r)
    best = min(res, key=lambda r: r["refactor_ms"] + r["solve_ms"])
    print(json.dumps({"config": args.config, "kind": "ablation" if args.ablation else "threshold sweep",
                      "results": res, "best": best["settings"]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
