"""The no-allocation solve entry point (``glu_solve_noalloc``) against
``glu_solve`` through the C ABI: same factors, same kernels, so the results
must agree to the parity bar (they are expected to be bitwise equal); two
calls in a row, the second one smaller, plus the capacity check."""

import numpy as np
import pytest
import scipy.sparse as sp

import circuitgen as cg
from paper_1908_00204_amd import glu

pytestmark = pytest.mark.gpu


def _solve_pair(A, nrhs, seed, dense_tail=0):
    import torch

    h = glu.Handle(device=0, dense_tail=dense_tail)
    h.analyze(A.n, A.colptr, A.rowind)
    h.factor(torch.from_numpy(A.values).cuda())
    b_host = cg.rhs(A.n, nrhs, seed)
    b = torch.from_numpy(np.ascontiguousarray(b_host.T)).cuda().t()
    x_ref = torch.empty((nrhs, A.n), dtype=torch.float64, device="cuda").t()
    x_na = torch.empty((nrhs, A.n), dtype=torch.float64, device="cuda").t()
    h.solve(b, x_ref)
    h.solve_noalloc(b, x_na)
    torch.cuda.synchronize()
    xr, xn = x_ref.cpu().numpy(), x_na.cpu().numpy()
    M = sp.csc_matrix((A.values, A.rowind, A.colptr), shape=(A.n, A.n))
    normA = abs(M).sum(axis=1).max()
    for c in range(nrhs):
        be = np.abs(M @ xn[:, c] - b_host[:, c]).max() / (normA * np.abs(xn[:, c]).max())
        assert be <= 1e-13, be
    rel = np.abs(xn - xr).max() / np.abs(xr).max()
    print(f"noalloc n={A.n} nrhs={nrhs} tail={h.query()['tail_m']} max rel diff vs glu_solve {rel:.2e}", flush=True)
    assert rel <= 1e-12
    return h, b


def test_noalloc_solve_matches_solve_twice_second_smaller():
    A1 = cg.circuit_matrix(20_000, rails=20, rail_frac=0.02, seed=71)
    _solve_pair(A1, 3, 571)
    A0 = cg.config_matrix("c0")
    _solve_pair(A0, 1, 500)


def test_noalloc_solve_without_dense_block():
    A = cg.circuit_matrix(5_000, rails=5, rail_frac=0.02, seed=72)
    _solve_pair(A, 2, 572, dense_tail=-1)


def test_noalloc_solve_rejects_oversized_requests():
    import torch

    A = cg.config_matrix("c0")
    h, _ = _solve_pair(A, 1, 500)
    cap = glu.Handle.noalloc_capacity()
    nrhs = cap // A.n  # 2 n nrhs alone exceeds the capacity
    b = torch.zeros((nrhs, A.n), dtype=torch.float64, device="cuda").t()
    with pytest.raises(glu.GluError) as ei:
        h.solve_noalloc(b, b)
    assert ei.value.code == glu.GLU_ERR_SCRATCH
