"""glu_batch: several factorizations whose sparse levels run as shared level
wavefronts (one launch per wavefront, replayed from a captured graph).  Every
handle must get bit for bit the factors it gets alone, within the oracle's
bar, in FP64 and in the mixed form."""

import numpy as np
import pytest
import scipy.sparse as sp

import circuitgen as cg
import oracle
from paper_1908_00204_amd import glu

pytestmark = pytest.mark.gpu


def _mats(k, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        n = int(round(np.exp(rng.uniform(np.log(1000), np.log(20000)))))
        rails = int(rng.integers(0, 6)) if i % 3 == 0 else 0
        out.append(cg.circuit_matrix(n, rails=rails, rail_frac=0.02 if rails else 0.0, seed=seed * 100 + i))
    return out


def _berr(A, x, b):
    M = sp.csc_matrix((A.values, A.rowind, A.colptr), shape=(A.n, A.n))
    normA = abs(M).sum(axis=1).max()
    x, b = x.reshape(A.n, -1), b.reshape(A.n, -1)
    return max(np.abs(M @ x[:, c] - b[:, c]).max() / (normA * np.abs(x[:, c]).max()) for c in range(x.shape[1]))


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_alone(precision):
    mats = _mats(8, 61 + precision)
    hs = []
    for A in mats:
        h = glu.Handle(device=0, precision=precision)
        h.analyze(A.n, A.colptr, A.rowind)
        hs.append(h)
    b = glu.Batch(hs)
    q = b.query()
    assert q["count"] == 8 and q["n_wavefronts"] > 0
    for rnd in range(3):  # graph replays, each checked against eager factorizations
        vals = [cg.perturbed_values(A.values, 7000 + 10 * rnd + i) for i, A in enumerate(mats)]
        b.factor(vals)
        for i, (A, h, v) in enumerate(zip(mats, hs, vals)):
            alone = glu.Handle(device=0, precision=precision, dense_gemm=1)  # the batch's bulk-update kernel
            alone.analyze(A.n, A.colptr, A.rowind)
            alone.factor(v)
            assert np.array_equal(h.export_factors(), alone.export_factors()), (rnd, i)
            Av = cg.CscMatrix(A.n, A.colptr, A.rowind, v)
            rhs = cg.rhs(A.n, 2, 7100 + i)
            assert _berr(Av, h.solve(rhs), rhs) <= 1e-13
    # the oracle on two of them (FP64 form: the 1e-12 bar)
    if precision == 0:
        for i in (0, 5):
            A = cg.CscMatrix(mats[i].n, mats[i].colptr, mats[i].rowind, vals[i])
            r = oracle.analyze(A, hs[i].export_symbolic()["perm"])
            lu = hs[i].export_factors()
            assert np.max(np.abs(lu - r.lu_val)) / np.max(np.abs(r.lu_val)) <= 1e-12
    b.close()


def test_batch_reports_the_failing_handle_and_state_errors():
    mats = _mats(3, 77)
    hs = []
    for A in mats:
        h = glu.Handle(device=0)
        h.analyze(A.n, A.colptr, A.rowind)
        hs.append(h)
    b = glu.Batch(hs)
    vals = [A.values.copy() for A in mats]
    vals[1][:] = 0.0  # every pivot of handle 1 is zero
    with pytest.raises(glu.GluError) as e:
        b.factor(vals)
    assert e.value.code == glu.GLU_ERR_ZERO_PIVOT
    assert hs[1].failed_column() >= 0
    vals[1] = mats[1].values.copy()
    b.factor(vals)  # all good again
    hs[2].analyze(mats[2].n, mats[2].colptr, mats[2].rowind)  # a new analysis invalidates the batch
    with pytest.raises(glu.GluError) as e:
        b.factor(vals)
    assert e.value.code == glu.GLU_ERR_STATE
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_solve_equals_solve_alone(precision):
    """glu_batch_solve runs every handle's solve (and, in the mixed form, its
    refinement rounds) concurrently; each handle's solution is bit for bit the
    one glu_solve gives it, and meets the backward-error bar."""
    import torch

    mats = _mats(6, 81 + precision)
    hs = []
    for A in mats:
        h = glu.Handle(device=0, precision=precision)
        h.analyze(A.n, A.colptr, A.rowind)
        hs.append(h)
    b = glu.Batch(hs)
    vals = [cg.perturbed_values(A.values, 8100 + i) for i, A in enumerate(mats)]
    b.factor(vals)
    dev = torch.device("cuda:0")
    rhs = [cg.rhs(A.n, 3, 8200 + i) for i, A in enumerate(mats)]
    bs = [torch.from_numpy(np.ascontiguousarray(r.T)).to(dev).t() for r in rhs]
    xs = b.solve(bs)
    torch.cuda.synchronize()
    iters = []
    for i, (A, h, v) in enumerate(zip(mats, hs, vals)):
        xb = xs[i].cpu().numpy()
        iters.append(h.query()["refine_iters"])
        xa = h.solve(rhs[i])
        assert np.array_equal(xb, xa), i
        Av = cg.CscMatrix(A.n, A.colptr, A.rowind, v)
        assert _berr(Av, xb, rhs[i]) <= 1e-13
    assert b.query()["t_solve_ms"] > 0
    if precision == 1:
        print("refinement steps per handle:", iters)
    with pytest.raises(ValueError):
        b.solve(bs[:-1])
    if precision == 1:
        with pytest.raises(glu.GluError):
            b.solve(bs, xs=bs)  # the mixed form's refinement re-reads b
    b.close()
