"""C-ABI tests that need no GPU: the library loads and exports every declared
symbol, host-side analysis (ordering, symbolic fill, relaxed DAG, levels)
matches the oracle bit for bit, and argument/state errors come back as codes."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import circuitgen as cg
import oracle
from paper_1908_00204_amd import glu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "glu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(glu_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(glu.EXPORTED)
    L = C.CDLL(glu.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_strerror_and_null_safety():
    L = glu.lib()
    for code in range(-8, 1):
        assert L.glu_strerror(code)
    L.glu_destroy(None)
    assert L.glu_failed_column(None) == -1


def _check_parity(A, h, perm=None):
    s = h.export_symbolic()
    r = oracle.analyze(A, s["perm"] if perm is None else perm, numeric=False)
    if perm is not None:
        assert np.array_equal(s["perm"], perm)
    for k in ("lu_colptr", "lu_rowind", "dag_ptr", "dag_idx", "level_ptr", "level_cols"):
        assert np.array_equal(s[k], getattr(r, k)), k
    q = h.query()
    st = oracle.level_stats(A.n, r.lu_colptr, r.lu_rowind, r.level_ptr, r.level_cols)
    assert q["nnz_lu"] == int(r.lu_colptr[-1])
    assert q["n_levels"] == len(r.level_ptr) - 1
    assert q["macs"] == st["macs"] and q["nnz_l"] == st["nL"] and q["nnz_u"] == st["nU"]
    return s, r


@pytest.mark.parametrize("ordering", [glu.GLU_ORDER_AMD, glu.GLU_ORDER_NATURAL])
def test_host_analysis_parity_c0(ordering):
    A = cg.config_matrix("c0")
    h = glu.Handle(device=-1, ordering=ordering)
    h.analyze(A.n, A.colptr, A.rowind)
    s, _ = _check_parity(A, h)
    if ordering == glu.GLU_ORDER_NATURAL:
        assert np.array_equal(s["perm"], np.arange(A.n))


@pytest.mark.parametrize("seed", range(8))
def test_host_analysis_parity_random(seed):
    n = [1, 2, 7, 40, 120, 300, 64, 500][seed]
    A = cg.random_pattern_matrix(n, min(0.5, 3.0 / n), 900 + seed, symmetric_pattern=(seed % 2 == 0))
    for ordering in (glu.GLU_ORDER_AMD, glu.GLU_ORDER_NATURAL):
        h = glu.Handle(device=-1, ordering=ordering)
        h.analyze(A.n, A.colptr, A.rowind)
        _check_parity(A, h)


def test_host_analysis_user_perm_and_rails():
    A = cg.circuit_matrix(3000, rails=5, rail_frac=0.05, seed=31)
    perm = oracle.mmd_order(A)
    h = glu.Handle(device=-1, ordering=glu.GLU_ORDER_USER)
    h.analyze(A.n, A.colptr, A.rowind, perm)
    _check_parity(A, h, perm)
    # rails (degree above 5 sqrt(n)) are ordered last by the AMD ordering
    h2 = glu.Handle(device=-1)
    h2.analyze(A.n, A.colptr, A.rowind)
    s = h2.export_symbolic()
    assert sorted(s["perm"][-5:].tolist()) == list(range(A.n - 5, A.n))
    _check_parity(A, h2)


def test_amd_is_a_valid_fill_reducing_permutation():
    A = cg.config_matrix("c0")
    h = glu.Handle(device=-1)
    h.analyze(A.n, A.colptr, A.rowind)
    s = h.export_symbolic()
    assert sorted(s["perm"].tolist()) == list(range(A.n))
    nat = glu.Handle(device=-1, ordering=glu.GLU_ORDER_NATURAL).analyze(A.n, A.colptr, A.rowind)
    mmd = glu.Handle(device=-1, ordering=glu.GLU_ORDER_USER).analyze(A.n, A.colptr, A.rowind,
                                                                    oracle.mmd_order(A))
    amd_nnz, nat_nnz, mmd_nnz = h.query()["nnz_lu"], nat.query()["nnz_lu"], mmd.query()["nnz_lu"]
    assert amd_nnz < 0.6 * nat_nnz
    assert amd_nnz < 1.2 * mmd_nnz


def test_argument_errors():
    h = glu.Handle(device=-1)
    with pytest.raises(glu.GluError) as e:
        h.query()
    assert e.value.code == glu.GLU_ERR_STATE
    # unsorted rows
    with pytest.raises(glu.GluError) as e:
        h.analyze(2, np.array([0, 2, 3]), np.array([1, 0, 1]))
    assert e.value.code == glu.GLU_ERR_ARG
    # duplicate rows
    with pytest.raises(glu.GluError) as e:
        h.analyze(2, np.array([0, 2, 3]), np.array([0, 0, 1]))
    assert e.value.code == glu.GLU_ERR_ARG
    # out of range
    with pytest.raises(glu.GluError) as e:
        h.analyze(2, np.array([0, 1, 2]), np.array([0, 2]))
    assert e.value.code == glu.GLU_ERR_ARG
    # bad user permutation
    hu = glu.Handle(device=-1, ordering=glu.GLU_ORDER_USER)
    with pytest.raises(glu.GluError) as e:
        hu.analyze(2, np.array([0, 1, 2]), np.array([0, 1]), np.array([0, 0]))
    assert e.value.code == glu.GLU_ERR_ARG
    with pytest.raises(glu.GluError) as e:
        hu.analyze(2, np.array([0, 1, 2]), np.array([0, 1]), None)
    assert e.value.code == glu.GLU_ERR_ARG
    # structurally singular: column 1 holds only row 0
    hn = glu.Handle(device=-1, ordering=glu.GLU_ORDER_NATURAL)
    with pytest.raises(glu.GluError) as e:
        hn.analyze(2, np.array([0, 1, 2]), np.array([0, 0]))
    assert e.value.code == glu.GLU_ERR_STRUCT_SINGULAR and e.value.column == 1
    # bad options
    with pytest.raises(glu.GluError) as e:
        glu.Handle(device=-1, ordering=7)
    assert e.value.code == glu.GLU_ERR_ARG


def test_host_only_handle_cannot_factor():
    A = cg.config_matrix("c0")
    h = glu.Handle(device=-1)
    h.analyze(A.n, A.colptr, A.rowind)
    with pytest.raises(glu.GluError) as e:
        h.factor(A.values)
    assert e.value.code == glu.GLU_ERR_DEVICE
    with pytest.raises(glu.GluError) as e:
        h.refactor(A.values)
    assert e.value.code == glu.GLU_ERR_STATE
    with pytest.raises(glu.GluError) as e:
        h.solve(np.ones(A.n))
    assert e.value.code == glu.GLU_ERR_STATE


@pytest.mark.parametrize("tail", [0, -1, 37])
def test_plan_covers_every_update(tail):
    """Every multiply-add of the factorization is planned exactly once, in
    aggregate: the products the sparse levels apply (targets outside the dense
    block), the Schur-complement update's (source before the block, target in
    it) and the block's own (source and target in it) add up to
    sum_j |L(:,j)| |U(j,:)|, each part counted here from the exported pattern;
    likewise the L / U entries of the columns / rows before the block."""
    A = cg.circuit_matrix(800, rails=2, rail_frac=0.1, seed=5)
    h = glu.Handle(device=-1, dense_tail=tail)
    h.analyze(A.n, A.colptr, A.rowind)
    q = h.query()
    s = h.export_symbolic()
    n, t = A.n, A.n - q["tail_m"]
    cp, ri = s["lu_colptr"], s["lu_rowind"]
    L = [ri[cp[j]:cp[j + 1]][ri[cp[j]:cp[j + 1]] > j] for j in range(n)]
    U = [[] for _ in range(n)]  # U(j,:) columns per row j
    for k in range(n):
        for j in ri[cp[k]:cp[k + 1]]:
            if j < k:
                U[j].append(k)
    lev = sch = blk = 0
    for j in range(n):
        for k in U[j]:
            for i in L[j]:
                if j >= t:
                    blk += 1
                elif i >= t and k >= t:
                    sch += 1
                else:
                    lev += 1
    assert q["level_macs"] == lev
    assert q["schur_macs"] == sch
    assert q["tail_macs"] == blk
    assert lev + sch + blk == q["macs"]
    assert q["level_nl"] == sum(len(L[j]) for j in range(t))
    assert q["level_nu"] == sum(len(U[j]) for j in range(t))
    assert q["n_tasks"] > 0 and q["n_work_items"] >= q["n_tasks"]
    assert sum(q["n_levels_mode"]) == q["n_exec_levels"] <= q["n_levels"]


def test_dense_tail_plan():
    """The executed levels are the levels restricted to the columns before the
    dense block, in order; the exported symbolic results do not change."""
    A = cg.config_matrix("c0")
    ref = glu.Handle(device=-1, dense_tail=-1).analyze(A.n, A.colptr, A.rowind)
    assert ref.query()["tail_m"] == 0
    for tail in (1, 100, 576, A.n):
        h = glu.Handle(device=-1, dense_tail=tail).analyze(A.n, A.colptr, A.rowind)
        q = h.query()
        assert q["tail_m"] == tail
        s, r = h.export_symbolic(), ref.export_symbolic()
        for k in s:
            assert np.array_equal(s[k], r[k]), k
        t = A.n - tail
        lp, lc = s["level_ptr"], s["level_cols"]
        expect = sum(1 for l in range(len(lp) - 1) if np.any(lc[lp[l]:lp[l + 1]] < t))
        assert q["n_exec_levels"] == expect
    auto = glu.Handle(device=-1).analyze(A.n, A.colptr, A.rowind).query()
    assert 0 <= auto["tail_m"] <= A.n


def test_gpu_analysis_option_is_refused():
    """The device DAG + levels step is switched off (its cause of a stall is
    not found); asking for it is an argument error, not a silent host run."""
    with pytest.raises(glu.GluError) as e:
        glu.Handle(device=-1, gpu_analysis=True)
    assert e.value.code == glu.GLU_ERR_ARG


def test_plan_is_the_same_on_any_number_of_host_threads():
    """The host level plan and Schur plan are built on several threads and
    concatenated in order: one thread and four give the same plan."""
    import json
    import subprocess
    import sys

    code = (
        "import json, circuitgen as cg\n"
        "from paper_1908_00204_amd import glu\n"
        "A = cg.circuit_matrix(20000, rails=20, rail_frac=0.02, seed=5150)\n"
        "h = glu.Handle(device=-1)\n"
        "h.analyze(A.n, A.colptr, A.rowind)\n"
        "q = h.query()\n"
        "print(json.dumps({k: q[k] for k in ('n_tasks', 'n_work_items', 'schur_steps', 'schur_tiles', 'schur_macs',"
        " 'macs', 'tail_m', 'n_exec_levels', 'n_solve_levels_l', 'n_solve_levels_u', 'level_macs')}))\n"
    )
    out = []
    for nt in ("1", "4"):
        env = dict(os.environ, GLU_PLAN_THREADS=nt, PYTHONPATH=ROOT)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT,
                           timeout=300)
        assert r.returncode == 0, r.stderr
        out.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert out[0] == out[1]
    assert out[0]["tail_m"] > 0 and out[0]["schur_tiles"] > 0
