"""Pins for the CPU oracle: each check compares the oracle with something other
than itself -- brute force on tiny inputs, closed forms, invariants, the
paper's worked-example facts, or an independent library routine -- so that a
dropped term, a wrong index or a transposed operand in the oracle fails here.
"""

import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import circuitgen as cg
import oracle
from oracle import right_looking as rl
from tests import _pins as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _csc_from_dense_pattern(F, values=None):
    cp, ri = pins.dense_pattern_to_csc(F)
    n = F.shape[0]
    if values is None:
        vals = np.ones(ri.size)
    else:
        vals = np.array([values[ri[p], j] for j in range(n) for p in range(cp[j], cp[j + 1])])
    return cg.CscMatrix(n, cp, ri, vals)


def _random_dominant(n, density, seed, symmetric=False):
    return cg.random_pattern_matrix(n, density, seed, symmetric_pattern=symmetric)


# ----------------------------------------------------------------------------- symbolic

@pytest.mark.parametrize("seed", range(12))
def test_symbolic_equals_boolean_elimination(seed):
    n = [5, 9, 17, 33, 64, 40][seed % 6]
    dens = [0.05, 0.1, 0.2, 0.3][seed % 4]
    A = _random_dominant(n, dens, seed, symmetric=(seed % 3 == 0))
    F = pins.csc_pattern_to_dense(n, A.colptr, A.rowind)
    cp, ri = oracle.symbolic(A)
    got = pins.csc_pattern_to_dense(n, cp, ri)
    assert np.array_equal(got, pins.boolean_elimination(F))


@pytest.mark.parametrize("seed", range(8))
def test_symbolic_fill_path_lemma(seed):
    n = 4 + seed
    A = _random_dominant(n, 0.25, 100 + seed)
    F = pins.csc_pattern_to_dense(n, A.colptr, A.rowind)
    cp, ri = oracle.symbolic(A)
    assert np.array_equal(pins.csc_pattern_to_dense(n, cp, ri), pins.fill_path(F))


@pytest.mark.parametrize("n", [1, 2, 7, 50])
def test_symbolic_closed_forms(n):
    eye = np.eye(n, dtype=bool)
    tri = eye | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    arrow_first = eye.copy(); arrow_first[0, :] = True; arrow_first[:, 0] = True
    arrow_last = eye.copy(); arrow_last[-1, :] = True; arrow_last[:, -1] = True
    for F, expect in [(eye, n), (tri, 3 * n - 2), (arrow_first, n * n), (arrow_last, 3 * n - 2)]:
        cp, ri = oracle.symbolic(_csc_from_dense_pattern(F))
        assert int(cp[-1]) == expect


def test_symbolic_structurally_singular():
    # B = [[1, 1], [0, 0]]: column 1 holds only row 0 and L(:,0) is empty, so
    # nothing can fill A_s(1,1)
    A = cg.CscMatrix(2, np.array([0, 1, 2], np.int64), np.array([0, 0], np.int32), np.ones(2))
    with pytest.raises(oracle.OracleError) as e:
        oracle.symbolic(A)
    assert e.value.code == oracle.ORC_ERR_STRUCT_SINGULAR and e.value.column == 1


def test_symbolic_fill_reaches_missing_diagonal():
    # B = [[1, 1], [1, 0]] structurally: (1,1) is created by eliminating 0
    A = cg.CscMatrix(2, np.array([0, 2, 3], np.int64), np.array([0, 1, 0], np.int32), np.ones(3))
    # column 1 has only row 0 -> its diagonal is reached through L(1,0)
    cp, ri = oracle.symbolic(A)
    assert list(ri[cp[1]:cp[2]]) == [0, 1]


def test_permute_roundtrip():
    A = _random_dominant(30, 0.15, 7)
    rng = np.random.default_rng(3)
    perm = rng.permutation(30).astype(np.int32)
    B = oracle.permute(A, perm)
    DA, DB = cg.to_dense(A), cg.to_dense(B)
    assert np.array_equal(DB, DA[np.ix_(perm, perm)])
    inv = np.argsort(perm).astype(np.int32)
    assert np.array_equal(cg.to_dense(oracle.permute(B, inv)), DA)


# ----------------------------------------------------------------------------- DAG + levels

def _golden_example():
    g = pins.parse_golden(os.path.join(GOLDEN, "paper_example_8x8.txt"))
    n = 8
    F = np.zeros((n, n), bool)
    for row in g["pattern"]:
        col = row[0] - 1
        for r in row[1:]:
            F[r - 1, col] = True
    return g, F


def test_paper_example_facts_hold():
    g, F = _golden_example()
    one = lambda i, j: F[i - 1, j - 1]  # noqa: E731  (1-based access)
    # F1
    assert [k for k in range(1, 7) if one(k, 7)] == [4, 6] and one(8, 7)
    # F2
    assert one(6, 4) and one(8, 4) and one(8, 6) and not one(7, 4) and not one(7, 6)
    # F3
    assert [k for k in range(4, 9) if one(3, k)] == [5, 8]
    # F4
    assert not any(one(k, 6) for k in range(1, 6))
    # the pattern is closed under fill
    assert np.array_equal(pins.boolean_elimination(F), F)
    # F5: double-U edges by the definition of Alg. 3 (strict bounds)
    du = set()
    for i in range(1, 9):
        for t in range(i + 1, 9):
            if not one(t, i):
                continue
            for j in range(t + 1, 9):
                if not one(j, t):
                    continue
                if any(one(i, k) and one(j, k) for k in range(t + 1, 9)):
                    du.add((i, t))
    assert du == {tuple(e) for e in g["double_u"]} == {(1, 2), (4, 6)}


def test_paper_example_dag_and_levels():
    g, F = _golden_example()
    n = 8
    A = _csc_from_dense_pattern(F)
    cp, ri = oracle.symbolic(A)
    assert np.array_equal(pins.csc_pattern_to_dense(n, cp, ri), F)
    dp, di = oracle.dag(n, cp, ri)
    got = {(i + 1, k + 1) for (i, k) in pins.edges_of(n, dp, di)}
    assert got == {tuple(e) for e in g["relaxed"]}
    # F5/F6: the relaxed DAG contains both double-U edges, the U-only one does not
    up, ui = rl.u_only_dag(n, cp, ri)
    uo = {(i + 1, k + 1) for (i, k) in pins.edges_of(n, up, ui)}
    assert uo == {tuple(e) for e in g["u_only"]}
    assert {(1, 2), (4, 6)} <= got and not ({(1, 2), (4, 6)} & uo)
    # F6: same levels as the exact DAG (GLU1.0 + double-U)
    lev, lp, lc = oracle.levels(n, dp, di)
    sets = [sorted(int(c) + 1 for c in lc[lp[l]:lp[l + 1]]) for l in range(len(lp) - 1)]
    assert sets == [sorted(s) for s in g["levels"]]
    exact = uo | {(1, 2), (4, 6)}
    eptr = np.zeros(n + 1, np.int64)
    eidx = []
    for k in range(1, n + 1):
        d = sorted(i for (i, kk) in exact if kk == k)
        eidx += [i - 1 for i in d]
        eptr[k] = len(eidx)
    lev2, lp2, lc2 = oracle.levels(n, eptr, np.array(eidx, np.int32))
    assert np.array_equal(lev, lev2)


def test_paper_example_u_only_levels_race():
    """Levels from the U-only DAG let column 6 read A_s(6,7) before column 4
    updates it (the double-U hazard): the level-by-level execution then differs
    from the sequential algorithm; with the relaxed DAG it is bitwise equal."""
    g, F = _golden_example()
    n = 8
    rng = np.random.default_rng(11)
    V = rng.uniform(0.5, 1.5, size=(n, n)) * F
    V[np.arange(n), np.arange(n)] += 4.0
    A = _csc_from_dense_pattern(F, V)
    cp, ri = oracle.symbolic(A)
    dp, di = oracle.dag(n, cp, ri)
    _, lp, lc = oracle.levels(n, dp, di)
    seq = rl.right_looking(n, cp, ri, A, order=lc)
    par = rl.levelized_right_looking(n, cp, ri, A, lp, lc)
    assert np.array_equal(seq, par)
    up, ui = rl.u_only_dag(n, cp, ri)
    _, ulp, ulc = oracle.levels(n, up, ui)
    bad = rl.levelized_right_looking(n, cp, ri, A, ulp, ulc)
    assert np.max(np.abs(bad - seq)) > 1e-3
    # the oracle (Alg. 1) agrees with the sequential right-looking result
    ref = oracle.factor(A, cp, ri)
    assert np.max(np.abs(ref - seq)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", range(10))
def test_dag_contains_exact_hazards(seed):
    n = [6, 10, 15, 24, 40][seed % 5]
    A = _random_dominant(n, 0.12 + 0.03 * (seed % 3), 200 + seed)
    cp, ri = oracle.symbolic(A)
    F = pins.csc_pattern_to_dense(n, cp, ri)
    dp, di = oracle.dag(n, cp, ri)
    E = pins.edges_of(n, dp, di)
    assert pins.exact_hazards(F) <= E


@pytest.mark.parametrize("seed", range(10))
def test_dag_second_traversal(seed):
    """Rebuild Alg. 4's edge set by scanning columns i and emitting i -> k for
    k in row i of U (when L(:,i) is not empty) and for k in L(:,i)."""
    n = [8, 20, 35, 50, 64][seed % 5]
    A = _random_dominant(n, 0.08, 300 + seed)
    cp, ri = oracle.symbolic(A)
    F = pins.csc_pattern_to_dense(n, cp, ri)
    E = set()
    for i in range(n):
        below = np.nonzero(F[i + 1:, i])[0] + i + 1
        if below.size:
            for k in np.nonzero(F[i, i + 1:])[0] + i + 1:
                E.add((i, int(k)))
        for k in below:
            E.add((i, int(k)))
    dp, di = oracle.dag(n, cp, ri)
    assert pins.edges_of(n, dp, di) == E
    # each list is sorted and unique
    for k in range(n):
        d = di[dp[k]:dp[k + 1]]
        assert np.all(np.diff(d) > 0)


@pytest.mark.parametrize("seed", range(10))
def test_levels_invariants(seed):
    n = [10, 30, 64, 100, 200][seed % 5]
    A = _random_dominant(n, 3.0 / n, 400 + seed)
    cp, ri = oracle.symbolic(A)
    dp, di = oracle.dag(n, cp, ri)
    lev, lp, lc = oracle.levels(n, dp, di)
    for (i, k) in pins.edges_of(n, dp, di):
        assert lev[i] < lev[k]
    for k in range(n):
        d = di[dp[k]:dp[k + 1]]
        if lev[k] == 0:
            assert d.size == 0
        else:
            assert np.any(lev[d] == lev[k] - 1)  # ASAP: tight
    assert sorted(lc.tolist()) == list(range(n))
    for l in range(len(lp) - 1):
        s = lc[lp[l]:lp[l + 1]]
        assert np.all(np.diff(s) > 0) and np.all(lev[s] == l)


@pytest.mark.parametrize("n", [1, 5, 33])
def test_levels_closed_forms(n):
    eye = np.eye(n, dtype=bool)
    tri = eye | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    arrow_last = eye.copy(); arrow_last[-1, :] = True; arrow_last[:, -1] = True
    blocks = eye.copy()
    for b in range(0, n - 1, 2):
        blocks[b:b + 2, b:b + 2] = True
    expect = {"eye": 1, "tri": n, "arrow": min(n, 2), "blocks": 2 if n > 1 else 1}
    for name, F in [("eye", eye), ("tri", tri), ("arrow", arrow_last), ("blocks", blocks)]:
        cp, ri = oracle.symbolic(_csc_from_dense_pattern(F))
        dp, di = oracle.dag(n, cp, ri)
        _, lp, _ = oracle.levels(n, dp, di)
        assert len(lp) - 1 == expect[name], name


@pytest.mark.parametrize("seed", range(6))
def test_levelized_executor_bitwise(seed):
    """The level-by-level executor equals sequential Alg. 2 in level order, bitwise."""
    n = [12, 25, 40][seed % 3]
    A = _random_dominant(n, 0.15, 500 + seed)
    cp, ri = oracle.symbolic(A)
    dp, di = oracle.dag(n, cp, ri)
    _, lp, lc = oracle.levels(n, dp, di)
    seq = rl.right_looking(n, cp, ri, A, order=lc)
    par = rl.levelized_right_looking(n, cp, ri, A, lp, lc)
    assert np.array_equal(seq, par)


# ----------------------------------------------------------------------------- numeric

def _split_lu(n, cp, ri, val):
    L = np.eye(n)
    U = np.zeros((n, n))
    for j in range(n):
        for p in range(cp[j], cp[j + 1]):
            i = ri[p]
            if i > j:
                L[i, j] = val[p]
            else:
                U[i, j] = val[p]
    return L, U


@pytest.mark.parametrize("seed", range(10))
def test_factor_vs_dense_doolittle(seed):
    n = [3, 8, 16, 31, 64][seed % 5]
    A = _random_dominant(n, 0.2, 600 + seed)
    cp, ri = oracle.symbolic(A)
    val = oracle.factor(A, cp, ri)
    L, U = _split_lu(n, cp, ri, val)
    Lr, Ur = pins.dense_doolittle(cg.to_dense(A))
    got = L + U - np.eye(n)
    ref = Lr + Ur - np.eye(n)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # entries outside the filled pattern are exactly zero in the dense factors
    F = pins.csc_pattern_to_dense(n, cp, ri)
    assert np.all(ref[~F] == 0.0)


@pytest.mark.parametrize("seed", range(4))
def test_factor_reconstruction_circuit(seed):
    A = cg.circuit_matrix(300 + 100 * seed, rails=2 * seed, rail_frac=0.05, seed=seed)
    perm = oracle.mmd_order(A)
    r = oracle.analyze(A, perm)
    L, U = _split_lu(A.n, r.lu_colptr, r.lu_rowind, r.lu_val)
    DB = cg.to_dense(r.B)
    assert np.max(np.abs(DB - L @ U)) <= 1e-13 * np.max(np.abs(DB))


def test_factor_special_cases():
    # diagonal: L = I, U = B
    n = 6
    D = np.diag(np.arange(1.0, n + 1))
    A = cg.from_dense(D)
    cp, ri = oracle.symbolic(A)
    assert np.array_equal(oracle.factor(A, cp, ri), np.arange(1.0, n + 1))
    # 2x2 closed form
    a, b, c, d = 3.0, 2.0, 5.0, 7.0
    A = cg.from_dense(np.array([[a, b], [c, d]]))
    cp, ri = oracle.symbolic(A)
    v = oracle.factor(A, cp, ri)
    # A_s order: col 0 = (0,0)=a, (1,0)=c/a ; col 1 = (0,1)=b, (1,1)=d - c/a*b
    assert v[0] == a and v[1] == c / a and v[2] == b and v[3] == d - (c / a) * b
    # tridiagonal: Thomas recurrence
    rng = np.random.default_rng(5)
    n = 40
    lo, di, up = rng.uniform(-1, 1, n), rng.uniform(3, 4, n), rng.uniform(-1, 1, n)
    T = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    A = cg.from_dense(T)
    cp, ri = oracle.symbolic(A)
    L, U = _split_lu(n, cp, ri, oracle.factor(A, cp, ri))
    d = np.zeros(n); l = np.zeros(n)
    d[0] = di[0]
    for i in range(1, n):
        l[i] = lo[i] / d[i - 1]
        d[i] = di[i] - l[i] * up[i - 1]
    assert np.allclose(np.diag(U), d, rtol=1e-14, atol=0)
    assert np.allclose(np.diag(L, -1), l[1:], rtol=1e-14, atol=0)


def test_factor_symmetric_and_spd():
    rng = np.random.default_rng(8)
    n = 30
    M = (rng.random((n, n)) < 0.15)
    M = M | M.T
    V = rng.uniform(-1, 1, (n, n)) * M
    S = (V + V.T) / 2
    S[np.arange(n), np.arange(n)] = np.abs(S).sum(axis=1) + 1.0
    A = cg.from_dense(S, pattern=M | np.eye(n, dtype=bool))
    cp, ri = oracle.symbolic(A)
    L, U = _split_lu(n, cp, ri, oracle.factor(A, cp, ri))
    Dg = np.diag(np.diag(U))
    assert np.max(np.abs(U - Dg @ L.T)) <= 1e-13 * np.max(np.abs(U))
    C = np.linalg.cholesky(S)
    assert np.max(np.abs(L @ np.sqrt(Dg) - C)) <= 1e-13 * np.max(np.abs(C))


@pytest.mark.parametrize("seed", range(4))
def test_factor_vs_superlu_natural(seed):
    A = cg.circuit_matrix(400, rails=3, rail_frac=0.05, seed=50 + seed)
    perm = oracle.mmd_order(A)
    B = oracle.permute(A, perm)
    cp, ri = oracle.symbolic(B)
    val = oracle.factor(B, cp, ri)
    M = sp.csc_matrix((B.values, B.rowind, B.colptr), shape=(B.n, B.n))
    lu = spla.splu(M, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    assert np.array_equal(lu.perm_r, np.arange(B.n)) and np.array_equal(lu.perm_c, np.arange(B.n))
    Ls = lu.L.toarray()
    Us = lu.U.toarray()
    L, U = _split_lu(B.n, cp, ri, val)
    scale = max(np.max(np.abs(Us)), 1.0)
    assert np.max(np.abs(L - Ls)) <= 1e-12
    assert np.max(np.abs(U - Us)) <= 1e-12 * scale


def test_right_looking_matches_left_looking():
    A = cg.circuit_matrix(120, rails=1, rail_frac=0.1, seed=9)
    r = oracle.analyze(A, oracle.mmd_order(A))
    seq = rl.right_looking(A.n, r.lu_colptr, r.lu_rowind, r.B)
    assert np.max(np.abs(seq - r.lu_val)) <= 1e-13 * np.max(np.abs(r.lu_val))


def test_zero_pivot_and_nonfinite():
    A = cg.from_dense(np.array([[1.0, 1.0], [1.0, 1.0]]))
    cp, ri = oracle.symbolic(A)
    with pytest.raises(oracle.OracleError) as e:
        oracle.factor(A, cp, ri)
    assert e.value.code == oracle.ORC_ERR_ZERO_PIVOT and e.value.column == 1
    A = cg.from_dense(np.array([[1.0, 2.0], [3.0, 4.0]]))
    A.values[1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.factor(A, *oracle.symbolic(A))
    assert e.value.code == oracle.ORC_ERR_NONFINITE


# ----------------------------------------------------------------------------- solve

@pytest.mark.parametrize("seed", range(4))
def test_solve_backward_error(seed):
    A = cg.circuit_matrix(500, rails=2, rail_frac=0.05, seed=70 + seed)
    perm = oracle.mmd_order(A)
    r = oracle.analyze(A, perm)
    b = cg.rhs(A.n, 3, 570 + seed)
    x = oracle.solve(r.lu_colptr, r.lu_rowind, r.lu_val, perm, b)
    M = sp.csc_matrix((A.values, A.rowind, A.colptr), shape=(A.n, A.n))
    normA = abs(M).sum(axis=1).max()
    for c in range(3):
        berr = np.abs(M @ x[:, c] - b[:, c]).max() / (normA * np.abs(x[:, c]).max())
        assert berr <= 1e-15
    xd = sla.solve(cg.to_dense(A), b)
    assert np.max(np.abs(x - xd)) <= 1e-8 * np.max(np.abs(xd))


def test_solve_closed_forms():
    n = 5
    D = np.diag([2.0, 4.0, 8.0, 0.5, 1.0])
    A = cg.from_dense(D)
    r = oracle.analyze(A)
    b = np.arange(1.0, n + 1)
    assert np.array_equal(oracle.solve(r.lu_colptr, r.lu_rowind, r.lu_val, r.perm, b), b / np.diag(D))
    # upper bidiagonal with unit diagonal: back substitution by hand
    Ub = np.eye(n) + np.diag(np.full(n - 1, 2.0), 1)
    A = cg.from_dense(Ub)
    r = oracle.analyze(A)
    b = np.ones(n)
    x = np.zeros(n)
    x[-1] = 1.0
    for i in range(n - 2, -1, -1):
        x[i] = 1.0 - 2.0 * x[i + 1]
    got = oracle.solve(r.lu_colptr, r.lu_rowind, r.lu_val, r.perm, b)
    assert np.array_equal(got, x)


def test_factor_extended_pins():
    """The extended-precision Alg. 1 agrees with the FP64 one to FP64 accuracy on
    well-conditioned inputs and reproduces exact small-integer factors."""
    A = _random_dominant(50, 0.1, 77)
    cp, ri = oracle.symbolic(A)
    v64 = oracle.factor(A, cp, ri)
    vx = oracle.factor_extended(A, cp, ri)
    assert np.max(np.abs(v64 - vx)) <= 1e-14 * np.max(np.abs(vx))
    # [[4, 2], [2, 3]] -> L = [[1, 0], [0.5, 1]], U = [[4, 2], [0, 2]], exact in binary
    A2 = cg.from_dense(np.array([[4.0, 2.0], [2.0, 3.0]]))
    cp2, ri2 = oracle.symbolic(A2)
    assert oracle.factor_extended(A2, cp2, ri2).tolist() == [4.0, 0.5, 2.0, 2.0]
    # against dense Doolittle in numpy's long double on a small circuit matrix
    Ac = cg.circuit_matrix(60, rails=1, rail_frac=0.3, seed=2)
    r = oracle.analyze(Ac, oracle.mmd_order(Ac), numeric=False)
    vx = oracle.factor_extended(r.B, r.lu_colptr, r.lu_rowind)
    D = cg.to_dense(r.B).astype(np.longdouble)
    n = D.shape[0]
    for kk in range(n):
        D[kk + 1:, kk] /= D[kk, kk]
        D[kk + 1:, kk + 1:] -= np.outer(D[kk + 1:, kk], D[kk, kk + 1:])
    ref = np.array([D[ri_, j] for j in range(n) for ri_ in r.lu_rowind[r.lu_colptr[j]:r.lu_colptr[j + 1]]],
                   dtype=np.float64)
    assert np.max(np.abs(vx - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_level_stats_hand_count_on_paper_example():
    """level_stats on the 8x8 example against counts done by hand from the
    golden pattern (1-based): L(:,j) sizes 1,1,1,2,0,1,1,0 -> nL = 7; U(j,:)
    sizes (row j) 1,1,2,1,1,1,1,0 -> nU = 8; multiply-adds
    sum_j |L(:,j)| |U(j,:)| = 1+1+2+2+0+1+1+0 = 8; four levels
    {1,3,4} {2,6} {5,7} {8}: widest 3; longest L column 2."""
    g, F = _golden_example()
    colptr, rowind = pins.dense_pattern_to_csc(F)
    lp = [0]
    lc = []
    for lev in g["levels"]:
        lc.extend(c - 1 for c in lev)
        lp.append(len(lc))
    st = oracle.level_stats(8, colptr, rowind, np.array(lp), np.array(lc))
    assert st == dict(nL=7, nU=8, macs=8, n_levels=4, widest=3, max_L=2)


@pytest.mark.parametrize("case", ["unsorted", "duplicate", "row_high", "row_negative", "colptr0",
                                  "colptr_decreasing"])
def test_oracle_rejects_malformed_csc(case):
    """The oracle's input check (CSC with rows strictly increasing inside each
    column, in range, colptr starting at 0 and nondecreasing) refuses each
    malformed input through both entry points that read a CSC."""
    cp, ri = {
        "unsorted": ([0, 2, 3], [1, 0, 1]),
        "duplicate": ([0, 2, 3], [0, 0, 1]),
        "row_high": ([0, 1, 2], [0, 2]),
        "row_negative": ([0, 1, 2], [-1, 1]),
        "colptr0": ([1, 2, 3], [0, 0, 1]),
        "colptr_decreasing": ([0, 2, 1], [0, 1]),
    }[case]
    cp = np.array(cp, np.int64)
    ri = np.array(ri, np.int32)
    A = cg.CscMatrix(2, cp, ri, np.ones(ri.size))
    with pytest.raises(oracle.OracleError):
        oracle.permute(A, np.arange(2))
    with pytest.raises(oracle.OracleError):
        oracle.symbolic(A)
    ok = cg.CscMatrix(2, np.array([0, 2, 4], np.int64), np.array([0, 1, 0, 1], np.int32), np.ones(4))
    oracle.permute(ok, np.arange(2))
    oracle.symbolic(ok)


@pytest.mark.parametrize("seed", range(6))
def test_fill_lemma_searches_match_brute_force_and_symbolic(seed):
    """oracle.fill_lower / fill_upper (one column's lower part, one row's upper
    part, from the fill-path lemma) against the brute-force path lemma on
    n <= 12 and against the reach-based symbolic pattern on larger inputs,
    including patterns with missing diagonals and unsymmetric structure."""
    rng = np.random.default_rng(4400 + seed)
    n = [6, 9, 12, 40, 120, 300][seed]
    F = rng.random((n, n)) < min(0.5, 3.0 / n)
    np.fill_diagonal(F, rng.random(n) < 0.8)
    # keep it structurally nonsingular: B(0,0) and the two off-diagonals put
    # every diagonal in the fill (column j+1 reaches j+1 through row j)
    F[0, 0] = True
    F[np.arange(1, n), np.arange(n - 1)] = True
    F[np.arange(n - 1), np.arange(1, n)] = True
    cp, ri = pins.dense_pattern_to_csc(F)
    B = cg.CscMatrix(n, cp, ri, np.ones(ri.size))
    try:
        lcp, lri = oracle.symbolic(B)
    except oracle.OracleError:
        pytest.skip("structurally singular draw")
    S = pins.csc_pattern_to_dense(n, lcp, lri)
    if n <= 12:
        assert np.array_equal(pins.fill_path(F), S)
    for j in range(n):
        assert np.array_equal(oracle.fill_lower(B, j), np.nonzero(S[j:, j])[0] + j)
        assert np.array_equal(oracle.fill_upper(B, j), np.nonzero(S[j, j:])[0] + j)
