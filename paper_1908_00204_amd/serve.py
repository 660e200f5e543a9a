"""Serving loop for Newton-iteration-like clients: refactor-and-solve requests
on resident patterns, continuous admission by device bytes, overlapped work.

The paper's motivating use is the repetition of the numeric factorization on a
fixed pattern inside Newton iterations (Section III, before III-A): the
symbolic analysis is done once and only the values change.  A server here
holds, for each pattern family, the analyzed pattern, its level plan and its
factor storage resident on the GPU (one or more handles of the C ABI), and
serves requests "refactor with these values, then solve these right-hand
sides".  Requests that arrive while others run are admitted as soon as a
worker is free and the device bytes they need fit the budget beside what is
already in flight (continuous batching: no request waits for a batch to
close), and the admitted requests run concurrently, each on its own HIP
stream, so their kernels overlap on the device.  Every computation runs in the
HIP library through the C ABI; this module only schedules calls.

Results do not depend on what else runs: every kernel of a request reads and
writes only its own handle's buffers, in a fixed order, so a request's factors
and solution are bitwise the same alone and in the mix (tested).

The benchmark serves the same request stream with plain FP64 handles and with
the mixed form (FP32 sparse levels, FP64 refinement in the solve), both at the
offered rate derived from the FP64 form's one-at-a-time capacity.

Usage (serving benchmark; prints one JSON line):
    python -m paper_1908_00204_amd.serve [--requests 200] [--rate-frac 0.7] [--forms fp64,mixed]
"""

from __future__ import annotations

import argparse
import collections
import json
import os
import queue
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import glu


@dataclass
class Request:
    family: int
    values: np.ndarray          # float64[nnz(A)] in the family's CSC order (host)
    rhs: np.ndarray             # float64 (n, nrhs), column-major (host)
    arrival: float = 0.0        # perf_counter() when submitted
    start: float = 0.0          # when admitted to a worker
    done: float = 0.0           # when its solution was back on the host
    x: np.ndarray | None = None
    error: str | None = None
    ticket: int = 0

    @property
    def latency_ms(self) -> float:
        return (self.done - self.arrival) * 1e3

    def device_bytes(self, n: int) -> int:
        """Device memory a request holds while it runs: its values, its
        right-hand sides and its solution."""
        return 8 * (self.values.size + 2 * n * self.rhs.shape[1])


@dataclass
class Family:
    """A resident pattern: analyzed once, its handles keep the plan and the
    factor storage on the device."""
    n: int
    colptr: np.ndarray
    rowind: np.ndarray
    handles: list = field(default_factory=list)
    free: collections.deque = field(default_factory=collections.deque)
    device_bytes: int = 0


class Server:
    """Continuous-batching request loop over resident pattern families.

    families: list of (n, colptr, rowind) patterns; replicas: handles per
    family (requests of one family run concurrently up to this many);
    workers: requests in flight at once (one host thread and one HIP stream
    each); budget_bytes: device bytes requests may hold in flight beside the
    resident families (admission control)."""

    def __init__(self, families, device: int = 0, workers: int = 4, replicas: int = 2,
                 budget_bytes: int = 8 << 30, handle_kw: dict | None = None):
        import torch

        self.device = device
        self.torch = torch
        self.budget = int(budget_bytes)
        self.fams: list[Family] = []
        for (n, cp, ri) in families:
            f = Family(n, np.asarray(cp, np.int64), np.asarray(ri, np.int32))
            for _ in range(replicas):
                h = glu.Handle(device=device, **(handle_kw or {}))
                h.analyze(n, f.colptr, f.rowind)
                f.handles.append(h)
                f.free.append(h)
                f.device_bytes += h.query()["device_bytes"]
            self.fams.append(f)
        self.resident_bytes = sum(f.device_bytes for f in self.fams)
        self._lock = threading.Condition()
        self._pending: collections.deque[Request] = collections.deque()
        self._inflight_bytes = 0
        self._stop = False
        self._done_q: queue.Queue = queue.Queue()
        self._count = 0
        self._threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(workers)]
        for t in self._threads:
            t.start()

    # ---- admission
    def submit(self, req: Request) -> None:
        req.arrival = time.perf_counter()
        with self._lock:
            self._count += 1
            req.ticket = self._count
            self._pending.append(req)
            self._lock.notify_all()

    def _admissible(self):
        """First pending request (arrival order) whose family has a free
        handle and whose bytes fit the budget; None if there is none."""
        for req in self._pending:
            f = self.fams[req.family]
            if f.free and self._inflight_bytes + req.device_bytes(f.n) <= self.budget:
                return req
            if not self._inflight_bytes and req.device_bytes(f.n) > self.budget:
                return req  # alone and still too big: run it anyway rather than stall forever
        return None

    def _worker(self):
        torch = self.torch
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(device=self.device)
        while True:
            with self._lock:
                req = None
                while not self._stop:
                    req = self._admissible()
                    if req is not None:
                        break
                    self._lock.wait(0.05)
                if self._stop and req is None:
                    return
                self._pending.remove(req)
                f = self.fams[req.family]
                h = f.free.popleft()
                nbytes = req.device_bytes(f.n)
                self._inflight_bytes += nbytes
            req.start = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    v = torch.from_numpy(req.values).to(f"cuda:{self.device}", non_blocking=False)
                    b = torch.from_numpy(np.ascontiguousarray(req.rhs.T)).to(f"cuda:{self.device}").t()
                    x = torch.empty((req.rhs.shape[1], f.n), dtype=torch.float64,
                                    device=f"cuda:{self.device}").t()
                    h.factor(v, stream=stream)
                    h.solve(b, x, stream=stream)
                    req.x = x.cpu().numpy()
            except Exception as e:  # the error is the request's result
                req.error = repr(e)
            req.done = time.perf_counter()
            with self._lock:
                f.free.append(h)
                self._inflight_bytes -= nbytes
                self._lock.notify_all()
            self._done_q.put(req)

    def wait(self, count: int, timeout: float = 600.0) -> list[Request]:
        """Collect `count` finished requests (completion order)."""
        out = []
        end = time.perf_counter() + timeout
        while len(out) < count:
            out.append(self._done_q.get(timeout=max(0.1, end - time.perf_counter())))
        return out

    def close(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        for t in self._threads:
            t.join(timeout=10)
        for f in self.fams:
            for h in f.handles:
                h.close()


def run_alone(server: Server, reqs: list[Request]) -> list[Request]:
    """Each request by itself, one after the other (the reference order)."""
    out = []
    for r in reqs:
        server.submit(r)
        out += server.wait(1)
    return out


def run_poisson(server: Server, reqs: list[Request], rate_per_s: float, seed: int = 0) -> list[Request]:
    """Submit the requests at Poisson arrival times of the given rate from this
    thread while the workers serve them; return them in completion order."""
    rng = np.random.default_rng(seed)
    t = time.perf_counter()
    for r in reqs:
        t += rng.exponential(1.0 / rate_per_s)
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)
        server.submit(r)
    return server.wait(len(reqs))


def summary(done: list[Request], wall_s: float) -> dict:
    lat = np.array([r.latency_ms for r in done])
    return {"requests": len(done), "errors": sum(r.error is not None for r in done),
            "throughput_req_s": len(done) / wall_s,
            "solves_per_s": sum(r.rhs.shape[1] for r in done) / wall_s,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_mean": float(lat.mean())}


def main() -> int:
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import circuitgen as cg

    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate-frac", type=float, default=0.7,
                    help="Poisson rate as a fraction of the measured one-at-a-time capacity")
    ap.add_argument("--sizes", default="5000,20000,50000,100000,200000,300000,400000,500000")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--forms", default="fp64,mixed",
                    help="comma list of fp64 (plain FP64 per request) and mixed (FP32 factor + FP64 refinement)")
    args = ap.parse_args()
    sizes = [int(s) for s in args.sizes.split(",")]
    rng = np.random.default_rng(4000)
    fams, bases = [], []
    for i, n in enumerate(sizes):
        rails = int(rng.integers(0, 201))
        A = cg.circuit_matrix(n, rails=rails, rail_frac=0.005 if rails else 0.0, seed=4000 + i)
        fams.append((A.n, A.colptr, A.rowind))
        bases.append(A)
        print(f"[serve] family {i}: n={n} rails={rails} nnz={A.nnz}", file=sys.stderr, flush=True)
    def make(k, seed):
        r = np.random.default_rng(seed)
        out = []
        for j in range(k):
            fi = int(r.integers(0, len(fams)))
            A = bases[fi]
            nrhs = int(r.integers(1, 9))
            out.append(Request(fi, cg.perturbed_values(A.values, seed=seed * 100000 + j),
                               cg.rhs(A.n, nrhs, seed * 100000 + j + 7)))
        return out

    forms = {"fp64": 0, "mixed": 1}
    res, rate = {}, None
    for name in args.forms.split(","):
        t0 = time.perf_counter()
        srv = Server(fams, workers=args.workers, replicas=2, handle_kw={"precision": forms[name]})
        print(f"[serve] {name}: {len(fams)} families resident ({srv.resident_bytes / 1e9:.2f} GB) in "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        # warm every handle once, then the one-at-a-time capacity
        for fi, A in enumerate(bases):
            for _ in range(2):
                srv.submit(Request(fi, A.values.copy(), cg.rhs(A.n, 1, 1)))
        srv.wait(2 * len(bases))
        cal = make(max(16, args.requests // 10), 1)
        t = time.perf_counter()
        run_alone(srv, cal)
        cap = len(cal) / (time.perf_counter() - t)
        print(f"[serve] {name}: one-at-a-time capacity {cap:.1f} requests/s", file=sys.stderr, flush=True)
        if rate is None:  # every form sees the first form's offered rate
            rate = args.rate_frac * cap * args.workers / 2
        reqs = make(args.requests, 2)
        t = time.perf_counter()
        done = run_poisson(srv, reqs, rate_per_s=rate, seed=3)
        wall = time.perf_counter() - t
        srv.close()
        res[name] = {"capacity_one_at_a_time_req_s": cap, **summary(done, wall)}
        print(f"[serve] {name}: {res[name]}", file=sys.stderr, flush=True)
    out = {"metric": "p50/p99 serve latency (refactor + solve requests)", "families": sizes,
           "workers": args.workers, "offered_rate_req_s": rate, **res}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
