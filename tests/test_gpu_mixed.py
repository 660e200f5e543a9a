"""The mixed-precision form (glu_options.precision = 1): FP32 factorization
of the sparse levels with FP32 arithmetic (a dense trailing block, when there
is one, in FP64 from the FP32 values), FP64 iterative refinement in the solve,
FP64 fallback.  Every result states its error against the FP64 oracle."""

import numpy as np
import pytest
import scipy.sparse as sp

import circuitgen as cg
import oracle
from paper_1908_00204_amd import glu

pytestmark = pytest.mark.gpu

BERR_TOL = 1e-13


def say(*a):
    import sys

    print(*a, file=sys.stderr, flush=True)


def berr(A, x, b):
    M = sp.csc_matrix((A.values, A.rowind, A.colptr), shape=(A.n, A.n))
    normA = abs(M).sum(axis=1).max()
    x = x.reshape(A.n, -1)
    b = b.reshape(A.n, -1)
    return max(np.abs(M @ x[:, c] - b[:, c]).max() / (normA * np.abs(x[:, c]).max()) for c in range(x.shape[1]))


def sparse_part(h, lu):
    """Factor entries of the columns before the dense block (all if none)."""
    q = h.query()
    if q["tail_m"] == 0:
        return lu
    t = q["n"] - q["tail_m"]
    return lu[: h.export_symbolic()["lu_colptr"][t]]


@pytest.mark.parametrize("tail", [0, -1])
@pytest.mark.parametrize("case", ["c0", "rails", "random"])
def test_fp32_factors_refined_to_fp64_accuracy(case, tail):
    if case == "c0":
        A = cg.config_matrix("c0")
    elif case == "rails":
        A = cg.circuit_matrix(20000, rails=20, rail_frac=0.02, seed=8801)
    else:
        A = cg.random_pattern_matrix(700, 0.01, 8802, symmetric_pattern=False)
    h = glu.Handle(device=0, precision=1, dense_tail=tail)
    h.analyze(A.n, A.colptr, A.rowind)
    h.factor(A.values)
    s = h.export_symbolic()
    r = oracle.analyze(A, s["perm"])
    for k in ("lu_colptr", "lu_rowind", "dag_ptr", "dag_idx", "level_ptr", "level_cols"):
        assert np.array_equal(s[k], getattr(r, k)), k
    lu32 = h.export_factors()
    e32 = np.max(np.abs(lu32 - r.lu_val)) / np.max(np.abs(r.lu_val))
    # FP32 factors: the sparse columns' values are exactly representable in FP32
    sp32 = sparse_part(h, lu32)
    assert np.array_equal(sp32.astype(np.float32).astype(np.float64), sp32)
    b = cg.rhs(A.n, 3, 8803)
    x = h.solve(b)
    q = h.query()
    be = berr(A, x, b)
    xo = oracle.solve(r.lu_colptr, r.lu_rowind, r.lu_val, r.perm, b)
    ex = np.max(np.abs(x - xo)) / np.max(np.abs(xo))
    say(f"mixed {case} (dense block {q['tail_m']}): FP32 factors vs FP64 oracle {e32:.2e}; refined x vs oracle x {ex:.2e}; "
        f"backward error {be:.2e} after {q['refine_iters']} steps, fallback {q['fp64_fallback']}")
    assert q["precision"] == 1
    assert e32 < 1e-3
    assert be <= BERR_TOL
    assert q["refine_berr"] <= BERR_TOL


def test_large_dense_block_in_fp32():
    """A dense block of 8,192 columns or more is factorized in FP32 in the
    mixed form (the library's no-pivot LU on an FP32 copy): every factor is
    then an FP32 value, and the refined solution meets the FP64 bar."""
    A = cg.circuit_matrix(20000, rails=20, rail_frac=0.02, seed=8801)
    h = glu.Handle(device=0, precision=1, dense_tail=8192)
    h.analyze(A.n, A.colptr, A.rowind)
    h.factor(A.values)
    q = h.query()
    assert q["tail_m"] == 8192
    lu = h.export_factors()
    assert np.array_equal(lu.astype(np.float32).astype(np.float64), lu)
    r = oracle.analyze(A, h.export_symbolic()["perm"])
    e32 = np.max(np.abs(lu - r.lu_val)) / np.max(np.abs(r.lu_val))
    b = cg.rhs(A.n, 2, 8806)
    x = h.solve(b)
    q = h.query()
    be = berr(A, x, b)
    say(f"mixed, FP32 dense block 8192: factors vs FP64 oracle {e32:.2e}; backward error {be:.2e} after "
        f"{q['refine_iters']} steps, fallback {q['fp64_fallback']}")
    assert e32 < 1e-2
    assert be <= BERR_TOL


def test_fp64_fallback_when_refinement_is_not_allowed():
    """With no refinement steps allowed the FP32 solve is not accurate enough,
    so the solve refactorizes in FP64 on the same plan and returns an FP64
    solution; the next factor goes back to FP32."""
    A = cg.config_matrix("c0")
    h = glu.Handle(device=0, precision=1, refine_max_iters=-1)
    h.analyze(A.n, A.colptr, A.rowind)
    h.factor(A.values)
    b = cg.rhs(A.n, 1, 8804)
    x = h.solve(b)
    q = h.query()
    assert q["fp64_fallback"] == 1 and q["refine_iters"] == 0
    assert berr(A, x, b) <= BERR_TOL
    lu = h.export_factors()
    r = oracle.analyze(A, h.export_symbolic()["perm"])
    assert np.max(np.abs(lu - r.lu_val)) / np.max(np.abs(r.lu_val)) <= 1e-12  # FP64 factors now
    v = cg.perturbed_values(A.values, 8805)
    h.refactor(v)
    lu32 = sparse_part(h, h.export_factors())
    assert np.array_equal(lu32.astype(np.float32).astype(np.float64), lu32)


def test_mixed_form_option_errors():
    with pytest.raises(glu.GluError):
        glu.Handle(device=0, precision=1, force_mode=glu.GLU_MODE_STREAM)
    with pytest.raises(glu.GluError):
        glu.Handle(device=0, precision=2)
