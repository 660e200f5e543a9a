/*
 * CPU oracle for the levelized sparse LU path.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  The product path never calls it and shares no code with
 * it.  It is deliberately plain and slow: single-threaded, no blocking, no
 * reordering beyond what each cited definition states, compiled with
 * -ffp-contract=off so every multiply and subtract is rounded separately.
 *
 * Notation (paper, Section II): A_s is the filled matrix holding L (strictly
 * below the diagonal, unit diagonal implied) and U (diagonal and above) in
 * place, A_s = L + U - I.  Everything here is 0-based; B = P A P^T with
 * B(i,j) = A(perm[i], perm[j]) (perm[new] = old) is the matrix that is
 * factorized without pivoting.
 *
 * Functions and the passage each follows:
 *   orc_permute   B = P A P^T                     (preprocessing, Section II-C)
 *   orc_symbolic  fill pattern of A_s by reachability in the graph of L
 *                 (the symbolic analysis done before Alg. 1, Section II-A)
 *   orc_dag       relaxed column dependencies, "look up" + "look left"
 *                 (Alg. 4, Section III-A)
 *   orc_levels    levelization: level(k) = 1 + max level of k's dependencies
 *                 (Section II-C, levels of mutually independent columns)
 *   orc_factor    Gilbert-Peierls left-looking numeric LU (Alg. 1, Section II-A)
 *   orc_solve     x = P^T U^-1 L^-1 P b, two sequential triangular solves
 *                 (Section I)
 *   orc_fill_lower, orc_fill_upper
 *                 the lower part of one column and the upper part of one row
 *                 of the fill pattern straight from the fill-path lemma (Rose
 *                 and Tarjan, 1978): (i, j) is filled iff the directed graph
 *                 of B holds a path i -> ... -> j whose inner vertices are all
 *                 smaller than min(i, j); a second, independent definition of
 *                 the symbolic result, cheap enough to check sampled columns
 *                 and rows of patterns too large for orc_symbolic
 *   orc_factor_extended
 *                 Alg. 1 again, accumulating in the C long double type (64-bit
 *                 significand on x86-64): an accuracy reference that is much
 *                 closer to the exact factors than any FP64 summation order,
 *                 used to tell rounding-order differences from errors
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_ZERO_PIVOT (-3)
#define ORC_ERR_STRUCT_SINGULAR (-4)
#define ORC_ERR_NOMEM (-5)
#define ORC_ERR_NONFINITE (-7)

void orc_free(void *p) { free(p); }

/* Growable int32 array. */
typedef struct {
    int32_t *a;
    int64_t n, cap;
} ivec;

static int ivec_push(ivec *v, int32_t x) {
    if (v->n == v->cap) {
        int64_t c = v->cap ? 2 * v->cap : 1024;
        int32_t *p = (int32_t *)realloc(v->a, (size_t)c * sizeof(int32_t));
        if (!p) return -1;
        v->a = p;
        v->cap = c;
    }
    v->a[v->n++] = x;
    return 0;
}

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Validate a CSC matrix: sorted strictly increasing rows, in range. */
int orc_check_csc(int32_t n, const int64_t *colptr, const int32_t *rowind) {
    if (n < 0 || !colptr) return ORC_ERR_ARG;
    if (colptr[0] != 0) return ORC_ERR_ARG;
    for (int32_t j = 0; j < n; j++) {
        if (colptr[j + 1] < colptr[j]) return ORC_ERR_ARG;
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            if (rowind[p] < 0 || rowind[p] >= n) return ORC_ERR_ARG;
            if (p > colptr[j] && rowind[p] <= rowind[p - 1]) return ORC_ERR_ARG;
        }
    }
    return ORC_OK;
}

/*
 * B = P A P^T, B(i,j) = A(perm[i], perm[j]).  Output arrays are caller-sized
 * (bcolptr n+1, browind/bval nnz(A)); rows sorted ascending.  bval may be NULL.
 */
int orc_permute(int32_t n, const int64_t *colptr, const int32_t *rowind, const double *val,
                const int32_t *perm, int64_t *bcolptr, int32_t *browind, double *bval) {
    if (orc_check_csc(n, colptr, rowind) != ORC_OK || !perm) return ORC_ERR_ARG;
    int32_t *pinv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!pinv) return ORC_ERR_NOMEM;
    for (int32_t i = 0; i < n; i++) pinv[i] = -1;
    for (int32_t i = 0; i < n; i++) {
        if (perm[i] < 0 || perm[i] >= n || pinv[perm[i]] != -1) {
            free(pinv);
            return ORC_ERR_ARG;
        }
        pinv[perm[i]] = i;
    }
    bcolptr[0] = 0;
    for (int32_t j = 0; j < n; j++) {
        int32_t oj = perm[j];
        int64_t len = colptr[oj + 1] - colptr[oj];
        int64_t base = bcolptr[j];
        bcolptr[j + 1] = base + len;
        /* insertion sort of (new row, value) pairs: columns are short */
        for (int64_t q = 0; q < len; q++) {
            int32_t r = pinv[rowind[colptr[oj] + q]];
            double v = val ? val[colptr[oj] + q] : 0.0;
            int64_t t = base + q;
            while (t > base && browind[t - 1] > r) {
                browind[t] = browind[t - 1];
                if (bval) bval[t] = bval[t - 1];
                t--;
            }
            browind[t] = r;
            if (bval) bval[t] = v;
        }
    }
    free(pinv);
    return ORC_OK;
}

/*
 * Symbolic fill of A_s for B factorized without pivoting.
 *
 * Column j of A_s is the set of nodes reachable from struct(B(:,j)) in the
 * directed graph with an edge r -> c for every c in struct(L(:,r)), r < j
 * (Gilbert and Peierls: the nonzeros of the solution of L x = B(:,j)).  Rows
 * <= j form U(:,j), rows > j form L(:,j).  Entries are kept even if they may
 * cancel numerically.  Plain work-list reachability, then a sort.
 *
 * lu_colptr: caller array of n+1.  *lu_rowind_out: malloc'ed (orc_free).
 * Returns nnz(A_s) >= 0, or ORC_ERR_STRUCT_SINGULAR with *bad_col set when a
 * diagonal entry is absent from the filled pattern.
 */
int64_t orc_symbolic(int32_t n, const int64_t *bcolptr, const int32_t *browind,
                     int64_t *lu_colptr, int32_t **lu_rowind_out, int32_t *bad_col) {
    *lu_rowind_out = NULL;
    if (bad_col) *bad_col = -1;
    if (orc_check_csc(n, bcolptr, browind) != ORC_OK) return ORC_ERR_ARG;
    ivec all = {0, 0, 0};
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *work = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *found = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!diag || !mark || !work || !found) {
        free(diag); free(mark); free(work); free(found);
        return ORC_ERR_NOMEM;
    }
    for (int32_t i = 0; i < n; i++) mark[i] = -1;
    lu_colptr[0] = 0;
    for (int32_t j = 0; j < n; j++) {
        int64_t nw = 0, nf = 0;
        for (int64_t p = bcolptr[j]; p < bcolptr[j + 1]; p++) {
            int32_t r = browind[p];
            if (mark[r] != j) { mark[r] = j; work[nw++] = r; }
        }
        while (nw > 0) {
            int32_t r = work[--nw];
            found[nf++] = r;
            if (r < j) {
                /* out-edges of r: struct(L(:,r)) = rows of column r after its diagonal */
                for (int64_t p = diag[r] + 1; p < lu_colptr[r + 1]; p++) {
                    int32_t c = all.a[p];
                    if (mark[c] != j) { mark[c] = j; work[nw++] = c; }
                }
            }
        }
        qsort(found, (size_t)nf, sizeof(int32_t), cmp_i32);
        diag[j] = -1;
        for (int64_t q = 0; q < nf; q++) {
            if (found[q] == j) diag[j] = lu_colptr[j] + q;
            if (ivec_push(&all, found[q])) {
                free(diag); free(mark); free(work); free(found); free(all.a);
                return ORC_ERR_NOMEM;
            }
        }
        lu_colptr[j + 1] = lu_colptr[j] + nf;
        if (diag[j] < 0) {
            if (bad_col) *bad_col = j;
            free(diag); free(mark); free(work); free(found); free(all.a);
            return ORC_ERR_STRUCT_SINGULAR;
        }
    }
    free(diag); free(mark); free(work); free(found);
    if (!all.a) all.a = (int32_t *)malloc(sizeof(int32_t));
    *lu_rowind_out = all.a;
    return lu_colptr[n];
}

/* position of the diagonal in every column of a filled pattern */
static int diag_positions(int32_t n, const int64_t *lp, const int32_t *li, int64_t *diag) {
    for (int32_t j = 0; j < n; j++) {
        diag[j] = -1;
        for (int64_t p = lp[j]; p < lp[j + 1]; p++)
            if (li[p] == j) diag[j] = p;
        if (diag[j] < 0) return -1;
    }
    return 0;
}

/*
 * Relaxed dependency detection (Alg. 4).  For every column k:
 *   look up:   i < k with A_s(i,k) != 0 whose L column (strictly below the
 *              diagonal) is not empty;
 *   look left: i < k with A_s(k,i) != 0, i.e. L(k,i) != 0.
 * dep(k) is the union as a set, sorted ascending.  An edge i -> k means column
 * k depends on column i.
 * dag_ptr: caller array n+1; *dag_idx_out malloc'ed.  Returns #edges.
 */
int64_t orc_dag(int32_t n, const int64_t *lp, const int32_t *li, int64_t *dag_ptr,
                int32_t **dag_idx_out) {
    *dag_idx_out = NULL;
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!diag) return ORC_ERR_NOMEM;
    if (diag_positions(n, lp, li, diag)) { free(diag); return ORC_ERR_STRUCT_SINGULAR; }
    /* row view of L: for row r, the columns i < r with L(r,i) != 0 (ascending i) */
    int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t nl = 0;
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = diag[i] + 1; p < lp[i + 1]; p++) { rp[li[p] + 1]++; nl++; }
    for (int32_t r = 0; r < n; r++) rp[r + 1] += rp[r];
    int32_t *rc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nl > 0 ? nl : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t r = 0; r < n; r++) { fill[r] = rp[r]; mark[r] = -1; }
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = diag[i] + 1; p < lp[i + 1]; p++) rc[fill[li[p]]++] = i;
    ivec out = {0, 0, 0};
    dag_ptr[0] = 0;
    for (int32_t k = 0; k < n; k++) {
        int64_t m = 0;
        /* look up: U part of column k, strictly above the diagonal */
        for (int64_t p = lp[k]; p < diag[k]; p++) {
            int32_t i = li[p];
            int lnonempty = (lp[i + 1] - 1) > diag[i];
            if (lnonempty && mark[i] != k) { mark[i] = k; tmp[m++] = i; }
        }
        /* look left: row k of L */
        for (int64_t q = rp[k]; q < rp[k + 1]; q++) {
            int32_t i = rc[q];
            if (mark[i] != k) { mark[i] = k; tmp[m++] = i; }
        }
        qsort(tmp, (size_t)m, sizeof(int32_t), cmp_i32);
        for (int64_t q = 0; q < m; q++) ivec_push(&out, tmp[q]);
        dag_ptr[k + 1] = dag_ptr[k] + m;
    }
    free(diag); free(rp); free(rc); free(fill); free(mark); free(tmp);
    if (!out.a) out.a = (int32_t *)malloc(sizeof(int32_t));
    *dag_idx_out = out.a;
    return dag_ptr[n];
}

/*
 * Levelization.  level(k) = 0 when k depends on nothing, else 1 + the largest
 * level among its dependencies; computed in increasing k (every dependency of
 * k is a smaller column).  Level sets list their columns in ascending order.
 * lev: n, level_ptr: n+1 (caller), level_cols: n.  Returns the number of levels.
 */
int32_t orc_levels(int32_t n, const int64_t *dag_ptr, const int32_t *dag_idx, int32_t *lev,
                   int32_t *level_ptr, int32_t *level_cols) {
    int32_t nlev = 0;
    for (int32_t k = 0; k < n; k++) {
        int32_t l = 0;
        for (int64_t p = dag_ptr[k]; p < dag_ptr[k + 1]; p++) {
            int32_t i = dag_idx[p];
            if (i >= k) return ORC_ERR_ARG;
            if (lev[i] + 1 > l) l = lev[i] + 1;
        }
        lev[k] = l;
        if (l + 1 > nlev) nlev = l + 1;
    }
    for (int32_t l = 0; l <= nlev; l++) level_ptr[l] = 0;
    for (int32_t k = 0; k < n; k++) level_ptr[lev[k] + 1]++;
    for (int32_t l = 0; l < nlev; l++) level_ptr[l + 1] += level_ptr[l];
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nlev > 0 ? nlev : 1));
    for (int32_t l = 0; l < nlev; l++) pos[l] = level_ptr[l];
    for (int32_t k = 0; k < n; k++) level_cols[pos[lev[k]]++] = k;
    free(pos);
    return nlev;
}

/*
 * Gilbert-Peierls left-looking numeric factorization (Alg. 1).
 *
 * For each column j, left to right: scatter B(:,j) into a dense work vector x;
 * for every k < j with A_s(k,j) != 0 in ascending k, and every i with
 * A_s(i,k) != 0 below k: x(i) -= A_s(i,k) * x(k); the entries of x at the
 * rows of column j become U(:,j) (rows <= j) and, divided by the pivot
 * A_s(j,j), L(:,j) (rows > j).  No pivoting.
 *
 * lu_val: caller array nnz(A_s), written in A_s order.  Returns ORC_OK, or
 * ORC_ERR_ZERO_PIVOT / ORC_ERR_NONFINITE with *bad_col set.
 */
int orc_factor(int32_t n, const int64_t *bcolptr, const int32_t *browind, const double *bval,
               const int64_t *lp, const int32_t *li, double *lu_val, int32_t *bad_col) {
    if (bad_col) *bad_col = -1;
    int64_t nnzb = bcolptr[n];
    for (int64_t p = 0; p < nnzb; p++)
        if (!isfinite(bval[p])) return ORC_ERR_NONFINITE;
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *x = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!diag || !x) { free(diag); free(x); return ORC_ERR_NOMEM; }
    if (diag_positions(n, lp, li, diag)) { free(diag); free(x); return ORC_ERR_STRUCT_SINGULAR; }
    for (int32_t j = 0; j < n; j++) {
        for (int64_t p = bcolptr[j]; p < bcolptr[j + 1]; p++) x[browind[p]] = bval[p];
        /* triangular solve with the columns on the left (ascending k) */
        for (int64_t q = lp[j]; q < diag[j]; q++) {
            int32_t k = li[q];
            double xk = x[k];
            for (int64_t p = diag[k] + 1; p < lp[k + 1]; p++) {
                double prod = lu_val[p] * xk;
                x[li[p]] = x[li[p]] - prod;
            }
        }
        for (int64_t q = lp[j]; q < lp[j + 1]; q++) lu_val[q] = x[li[q]];
        double piv = lu_val[diag[j]];
        if (piv == 0.0 || !isfinite(piv)) {
            if (bad_col) *bad_col = j;
            free(diag); free(x);
            return ORC_ERR_ZERO_PIVOT;
        }
        for (int64_t q = diag[j] + 1; q < lp[j + 1]; q++) lu_val[q] = lu_val[q] / piv;
        for (int64_t q = lp[j]; q < lp[j + 1]; q++) x[li[q]] = 0.0;
    }
    free(diag); free(x);
    return ORC_OK;
}

/*
 * Solve A x = b with the factors of B = P A P^T: c = P b (c(i) = b(perm[i])),
 * forward substitution with unit-lower L, backward substitution with U, then
 * x(perm[i]) = c(i).  Column-oriented, sequential.  b and x are n x nrhs
 * column-major with leading dimensions ldb / ldx.
 */
int orc_solve(int32_t n, const int64_t *lp, const int32_t *li, const double *lu_val,
              const int32_t *perm, int32_t nrhs, const double *b, int64_t ldb, double *x,
              int64_t ldx) {
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!diag || !c) { free(diag); free(c); return ORC_ERR_NOMEM; }
    if (diag_positions(n, lp, li, diag)) { free(diag); free(c); return ORC_ERR_STRUCT_SINGULAR; }
    for (int32_t r = 0; r < nrhs; r++) {
        for (int32_t i = 0; i < n; i++) c[i] = b[(int64_t)r * ldb + perm[i]];
        for (int32_t j = 0; j < n; j++) {
            double cj = c[j];
            for (int64_t p = diag[j] + 1; p < lp[j + 1]; p++) c[li[p]] = c[li[p]] - lu_val[p] * cj;
        }
        for (int32_t j = n - 1; j >= 0; j--) {
            c[j] = c[j] / lu_val[diag[j]];
            double cj = c[j];
            for (int64_t p = lp[j]; p < diag[j]; p++) c[li[p]] = c[li[p]] - lu_val[p] * cj;
        }
        for (int32_t i = 0; i < n; i++) x[(int64_t)r * ldx + perm[i]] = c[i];
    }
    free(diag); free(c);
    return ORC_OK;
}

/*
 * Alg. 1 in extended precision: the same steps as orc_factor with a long
 * double work vector and long double factor entries, rounded to double only
 * on output.  Returns ORC_OK or ORC_ERR_ZERO_PIVOT (*bad_col set).
 */
int orc_factor_extended(int32_t n, const int64_t *bcolptr, const int32_t *browind, const double *bval,
                        const int64_t *lp, const int32_t *li, double *lu_val, int32_t *bad_col) {
    if (bad_col) *bad_col = -1;
    int64_t nnz = lp[n];
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    long double *x = (long double *)calloc((size_t)(n > 0 ? n : 1), sizeof(long double));
    long double *v = (long double *)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(long double));
    if (!diag || !x || !v) { free(diag); free(x); free(v); return ORC_ERR_NOMEM; }
    if (diag_positions(n, lp, li, diag)) { free(diag); free(x); free(v); return ORC_ERR_STRUCT_SINGULAR; }
    for (int32_t j = 0; j < n; j++) {
        for (int64_t p = bcolptr[j]; p < bcolptr[j + 1]; p++) x[browind[p]] = bval[p];
        for (int64_t q = lp[j]; q < diag[j]; q++) {
            int32_t k = li[q];
            long double xk = x[k];
            for (int64_t p = diag[k] + 1; p < lp[k + 1]; p++) x[li[p]] = x[li[p]] - v[p] * xk;
        }
        for (int64_t q = lp[j]; q < lp[j + 1]; q++) v[q] = x[li[q]];
        long double piv = v[diag[j]];
        if (piv == 0.0L) {
            if (bad_col) *bad_col = j;
            free(diag); free(x); free(v);
            return ORC_ERR_ZERO_PIVOT;
        }
        for (int64_t q = diag[j] + 1; q < lp[j + 1]; q++) v[q] = v[q] / piv;
        for (int64_t q = lp[j]; q < lp[j + 1]; q++) x[li[q]] = 0.0L;
    }
    for (int64_t q = 0; q < nnz; q++) lu_val[q] = (double)v[q];
    free(diag); free(x); free(v);
    return ORC_OK;
}



/*
 * Fill-path searches.  The directed graph of B has an edge u -> v iff
 * B(u,v) != 0.  orc_fill_lower(j): every i >= j with a path i -> ... -> j
 * whose inner vertices are below j, i.e. the rows of column j of A_s on and
 * below the diagonal; found by a backward search from j (the predecessors of
 * v are the rows of column v), expanding only vertices below j.
 * orc_fill_upper(i): every k >= i with a path i -> ... -> k whose inner
 * vertices are below i, i.e. the columns of row i of A_s on and right of the
 * diagonal; a forward search from i (the successors of u are the columns
 * holding row u), expanding only vertices below i.  The diagonal is in the
 * result iff B has it or a cycle through smaller vertices returns to it.
 * out: caller buffer of n int32, filled ascending; returns the count, or a
 * negative code.
 */
static int32_t fill_search(int32_t n, const int64_t *adj_ptr, const int32_t *adj, int32_t start, int32_t *out) {
    int32_t *mark = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!mark || !stack) {
        free(mark);
        free(stack);
        return ORC_ERR_NOMEM;
    }
    int32_t top = 0;
    stack[top++] = start;
    int started = 0;
    while (top > 0) {
        int32_t v = stack[--top];
        /* the start vertex is expanded once; any other vertex only if below start */
        if (v == start) {
            if (started) continue;
            started = 1;
        } else if (v > start) {
            continue;
        }
        for (int64_t p = adj_ptr[v]; p < adj_ptr[v + 1]; p++) {
            int32_t u = adj[p];
            if (mark[u]) continue;
            mark[u] = 1;
            if (u < start) stack[top++] = u;
        }
    }
    int32_t cnt = 0;
    for (int32_t i = start; i < n; i++)
        if (mark[i]) out[cnt++] = i;
    free(mark);
    free(stack);
    return cnt;
}

int32_t orc_fill_lower(int32_t n, const int64_t *bcolptr, const int32_t *browind, int32_t j, int32_t *out) {
    if (orc_check_csc(n, bcolptr, browind) != ORC_OK || j < 0 || j >= n || !out) return ORC_ERR_ARG;
    return fill_search(n, bcolptr, browind, j, out);
}

int32_t orc_fill_upper(int32_t n, const int64_t *bcolptr, const int32_t *browind, int32_t i, int32_t *out) {
    if (orc_check_csc(n, bcolptr, browind) != ORC_OK || i < 0 || i >= n || !out) return ORC_ERR_ARG;
    /* rows of B as lists of columns (successors) */
    int64_t nnz = bcolptr[n];
    int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *rc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!rp || !rc) {
        free(rp);
        free(rc);
        return ORC_ERR_NOMEM;
    }
    for (int64_t p = 0; p < nnz; p++) rp[browind[p] + 1]++;
    for (int32_t r = 0; r < n; r++) rp[r + 1] += rp[r];
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!f) {
        free(rp);
        free(rc);
        return ORC_ERR_NOMEM;
    }
    for (int32_t r = 0; r < n; r++) f[r] = rp[r];
    for (int32_t c = 0; c < n; c++)
        for (int64_t p = bcolptr[c]; p < bcolptr[c + 1]; p++) rc[f[browind[p]]++] = c;
    int32_t cnt = fill_search(n, rp, rc, i, out);
    free(f);
    free(rp);
    free(rc);
    return cnt;
}
