"""The preprocessing flow of Section II-C on a matrix that needs it: a circuit
matrix with its rows shuffled and its rows and columns badly scaled has no
usable diagonal; glu_mc64's row permutation and scalings give one, and the
GPU factorization of the scaled, permuted matrix matches the oracle's and
solves the original system."""

import sys

import numpy as np
import pytest
import scipy.sparse as sp

import circuitgen as cg
import oracle
from paper_1908_00204_amd import glu

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_csc(M):
    M = sp.csc_matrix(M)
    M.sort_indices()
    return cg.CscMatrix(M.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.copy())


@pytest.mark.parametrize("n,seed", [(3000, 41), (20000, 42)])
def test_mc64_then_factor_and_solve(n, seed):
    say(f"mc64 n={n} seed={seed}")
    base = cg.circuit_matrix(n, seed=seed)
    rng = np.random.default_rng(seed)
    sigma = rng.permutation(n)
    r = 10.0 ** rng.uniform(-4, 4, n)
    c = 10.0 ** rng.uniform(-4, 4, n)
    B = sp.csc_matrix((base.values, base.rowind, base.colptr), shape=(n, n))
    A = to_csc(sp.diags(r) @ B[sigma, :] @ sp.diags(c))
    # without static pivoting the shuffled diagonal is missing
    h0 = glu.Handle(device=0)
    with pytest.raises(glu.GluError) as e:
        h0.analyze(A.n, A.colptr, A.rowind)
        h0.factor(A.values)
    assert e.value.code in (glu.GLU_ERR_STRUCT_SINGULAR, glu.GLU_ERR_ZERO_PIVOT)
    h0.close()

    perm, dr, dc = glu.mc64(A.n, A.colptr, A.rowind, A.values)
    As = sp.csc_matrix((A.values, A.rowind, A.colptr), shape=(n, n))
    M = to_csc((sp.diags(dr) @ As @ sp.diags(dc))[perm, :])
    assert np.all(np.abs(M.values) <= 1.0 + 1e-12)

    h = glu.Handle(device=0)
    h.analyze(M.n, M.colptr, M.rowind)
    h.factor(M.values)
    s = h.export_symbolic()
    ro = oracle.analyze(M, s["perm"])
    for k in ("lu_colptr", "lu_rowind", "dag_ptr", "dag_idx", "level_ptr", "level_cols"):
        assert np.array_equal(s[k], getattr(ro, k)), k
    lu = h.export_factors()
    assert np.max(np.abs(lu - ro.lu_val)) <= 1e-12 * np.max(np.abs(ro.lu_val))

    b = cg.rhs(n, 2, seed + 1)
    rhs_m = np.asfortranarray((dr[:, None] * b)[perm, :])
    y = h.solve(rhs_m)
    x = dc[:, None] * y
    Ms = sp.csc_matrix((M.values, M.rowind, M.colptr), shape=(n, n))
    normM = abs(Ms).sum(axis=1).max()
    for k in range(x.shape[1]):
        # normwise on the scaled system (entries <= 1), componentwise on A
        # itself (normwise figures mean little once rows differ by 10^8)
        bm = np.abs(Ms @ y[:, k] - rhs_m[:, k]).max() / (normM * np.abs(y[:, k]).max())
        cw = np.max(np.abs(As @ x[:, k] - b[:, k]) / (abs(As) @ np.abs(x[:, k]) + np.abs(b[:, k])))
        say(f"  column {k}: scaled-system backward error {bm:.2e}, componentwise on A {cw:.2e}")
        assert bm <= 1e-13
        assert cw <= 1e-11
    h.close()
