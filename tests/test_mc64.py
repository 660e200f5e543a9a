"""glu_mc64 (static pivoting and scaling of the preprocessing flow, Section
II-C) on the host: the matching maximizes the product of matched magnitudes
(brute force over every permutation on tiny inputs, scipy's minimum-weight
full bipartite matching on larger ones), the scalings certify it (all scaled
magnitudes <= 1, matched ones 1: the dual bound of the assignment problem),
and the error cases come back as codes."""

import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import min_weight_full_bipartite_matching

from paper_1908_00204_amd import glu


def hidden_matching_matrix(n, extra, seed, spread=6.0):
    """Sparse A with a perfect matching on a random row permutation, no
    diagonal preference, magnitudes spread over 10^+-spread/2 and random
    signs; `extra` more random entries per column."""
    rng = np.random.default_rng(seed)
    sigma = rng.permutation(n)
    rows = [sigma]
    cols = [np.arange(n)]
    for _ in range(extra):
        rows.append(rng.integers(0, n, n))
        cols.append(np.arange(n))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = rng.choice([-1.0, 1.0], r.size) * 10.0 ** rng.uniform(-spread / 2, spread / 2, r.size)
    A = sp.csc_matrix((v, (r, c)), shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    return A


def run_mc64(A):
    A = sp.csc_matrix(A)
    A.sort_indices()
    return glu.mc64(A.shape[0], A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data)


def log_product(A, row_of_col):
    D = A.toarray()
    return float(np.sum(np.log(np.abs(D[row_of_col, np.arange(A.shape[0])]))))


def check_certificate(A, perm, dr, dc, tol=1e-12):
    n = A.shape[0]
    assert sorted(perm.tolist()) == list(range(n)), "not a permutation"
    S = sp.diags(dr) @ A @ sp.diags(dc)
    assert np.abs(S.data).max() <= 1.0 + tol
    matched = np.abs(S.toarray()[perm, np.arange(n)]) if n <= 400 else \
        np.abs(np.asarray(S.tocsc()[perm, :].diagonal()))
    np.testing.assert_allclose(matched, 1.0, rtol=0, atol=tol)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_tiny(seed):
    n = 2 + seed % 5
    A = hidden_matching_matrix(n, 2, 100 + seed)
    perm, dr, dc = run_mc64(A)
    D = A.toarray()
    best = -np.inf
    for p in itertools.permutations(range(n)):
        vals = np.abs(D[list(p), np.arange(n)])
        if np.all(vals > 0):
            best = max(best, float(np.sum(np.log(vals))))
    assert abs(log_product(A, perm) - best) <= 1e-12 * max(1.0, abs(best))
    check_certificate(A, perm, dr, dc)


@pytest.mark.parametrize("n,extra,seed", [(300, 3, 1), (2000, 4, 2), (5000, 2, 3)])
def test_against_scipy_assignment(n, extra, seed):
    A = hidden_matching_matrix(n, extra, seed)
    perm, dr, dc = run_mc64(A)
    # minimum of sum(-log|a|) over perfect matchings, by scipy
    W = A.copy()
    W.data = 1.0 + np.log(np.abs(A.data).max()) - np.log(np.abs(W.data))  # positive weights
    W = sp.csr_matrix(W)
    rows, cols = min_weight_full_bipartite_matching(W)
    ref = np.empty(n, np.int64)
    ref[cols] = rows
    lp, lref = log_product(A, perm), log_product(A, ref)
    assert abs(lp - lref) <= 1e-10 * max(1.0, abs(lref))
    check_certificate(A, perm, dr, dc, tol=1e-10)


def test_dominant_matrix_keeps_identity():
    n = 50
    rng = np.random.default_rng(7)
    A = sp.random(n, n, density=0.1, random_state=8, format="csc")
    A = A + sp.diags(10.0 + np.abs(A).sum(axis=0).A1)
    A = sp.csc_matrix(A)
    perm, _, _ = run_mc64(A)
    assert np.array_equal(perm, np.arange(n))
    del rng


def test_empty_and_errors():
    perm, dr, dc = glu.mc64(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert perm.size == 0 and dr.size == 0 and dc.size == 0
    # two columns whose only rows coincide: no perfect matching
    A = sp.csc_matrix(np.array([[1.0, 2.0, 0.0], [0.0, 0.0, 3.0], [0.0, 0.0, 4.0]]))
    with pytest.raises(glu.GluError) as e:
        run_mc64(A)
    assert e.value.code == glu.GLU_ERR_STRUCT_SINGULAR
    # an all-zero (explicitly stored) column
    Z = sp.csc_matrix((np.array([1.0, 0.0]), np.array([0, 1]), np.array([0, 1, 2])), shape=(2, 2))
    with pytest.raises(glu.GluError) as e:
        run_mc64(Z)
    assert e.value.code == glu.GLU_ERR_STRUCT_SINGULAR
    N = sp.csc_matrix(np.array([[np.nan, 1.0], [1.0, 1.0]]))
    with pytest.raises(glu.GluError) as e:
        run_mc64(N)
    assert e.value.code == glu.GLU_ERR_NONFINITE_INPUT
    # unsorted rows within a column
    with pytest.raises(glu.GluError) as e:
        glu.mc64(2, np.array([0, 2, 3], np.int64), np.array([1, 0, 1], np.int32), np.ones(3))
    assert e.value.code == glu.GLU_ERR_ARG


def test_explicit_zeros_are_never_matched():
    # the only nonzero choice puts a(1,0) and a(0,1) on the diagonal
    A = sp.csc_matrix((np.array([0.0, 2.0, 3.0, 0.0]), np.array([0, 1, 0, 1]), np.array([0, 2, 4])), shape=(2, 2))
    perm, dr, dc = run_mc64(A)
    assert perm.tolist() == [1, 0]
    check_certificate(A, perm, dr, dc)
