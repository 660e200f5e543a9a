"""The serving loop (continuous admission over resident pattern families):
every request's solution is the same alone and in the concurrent mix, the
byte budget is respected, and every request finishes."""

import numpy as np
import pytest
import scipy.sparse as sp

import circuitgen as cg
from paper_1908_00204_amd import serve

pytestmark = pytest.mark.gpu


def _families():
    out = []
    for i, (n, rails) in enumerate([(3000, 0), (8000, 8), (20000, 20)]):
        out.append(cg.circuit_matrix(n, rails=rails, rail_frac=0.01 if rails else 0.0, seed=9100 + i))
    return out


def _requests(bases, k, seed):
    r = np.random.default_rng(seed)
    reqs = []
    for j in range(k):
        fi = int(r.integers(0, len(bases)))
        A = bases[fi]
        reqs.append(serve.Request(fi, cg.perturbed_values(A.values, seed=seed * 1000 + j),
                                  cg.rhs(A.n, int(r.integers(1, 5)), seed * 1000 + j + 1)))
    return reqs


@pytest.mark.parametrize("precision", [0, 1])
def test_same_result_alone_and_in_the_mix(precision):
    """Plain FP64 handles and the mixed form (FP32 sparse levels, FP64
    refinement): the same request gives the same bits alone and in the mix."""
    bases = _families()
    srv = serve.Server([(A.n, A.colptr, A.rowind) for A in bases], workers=4, replicas=2,
                       handle_kw={"precision": precision})
    try:
        alone = serve.run_alone(srv, _requests(bases, 24, 5))
        mix = serve.run_poisson(srv, _requests(bases, 24, 5), rate_per_s=5000.0, seed=1)
    finally:
        srv.close()
    by_key = {}
    for r in alone:
        assert r.error is None, r.error
        by_key[(r.family, r.values.tobytes()[:64], r.rhs.shape[1])] = r
    assert len(mix) == 24
    for r in mix:
        assert r.error is None, r.error
        ref = by_key[(r.family, r.values.tobytes()[:64], r.rhs.shape[1])]
        assert np.array_equal(r.x, ref.x)
        A = bases[r.family]
        M = sp.csc_matrix((r.values, A.rowind, A.colptr), shape=(A.n, A.n))
        normA = abs(M).sum(axis=1).max()
        for c in range(r.rhs.shape[1]):
            be = np.abs(M @ r.x[:, c] - r.rhs[:, c]).max() / (normA * np.abs(r.x[:, c]).max())
            assert be <= 1e-13
    # overlapping work: some requests started before others finished
    spans = sorted((r.start, r.done) for r in mix)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))


def test_admission_budget_holds_requests_back():
    """With a budget that fits the largest request alone, the loop still
    serves every request, and the requests in flight together never hold more
    bytes than the budget (a request's [start, done) lies inside the span in
    which its bytes are counted)."""
    bases = _families()[:2]
    reqs = _requests(bases, 10, 7)
    nbytes = {id(r): r.device_bytes(bases[r.family].n) for r in reqs}
    one = max(nbytes.values())
    srv = serve.Server([(A.n, A.colptr, A.rowind) for A in bases], workers=4, replicas=2, budget_bytes=one)
    try:
        done = serve.run_poisson(srv, reqs, rate_per_s=10000.0, seed=2)
    finally:
        srv.close()
    assert len(done) == 10 and all(r.error is None for r in done)
    for r in done:
        held = sum(nbytes[id(o)] for o in done if o.start <= r.start < o.done)
        assert held <= one, (held, one)
