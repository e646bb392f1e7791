/*
 * Reference oracle for SpTRSV on equation-rewritten DAGs -- TEST
 * INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, obviously-correct CPU implementation in FP64 of what
 * the GPU library computes: level-set analysis, equation rewriting, forward
 * substitution and its adjoint.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load this file's shared object.
 * It shares no code, header or table with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared oracle.c -o liboracle.so
 * (-ffp-contract=off: every multiply and subtract below is rounded
 * separately, in the order written.)
 *
 * Storage: CSR with int32 row pointers and column indices; inside a row the
 * columns strictly ascend and the diagonal is the last entry.  Dense blocks
 * of k right-hand sides are column-major with a leading dimension >= n.
 *
 * Parity pins (what checks this file against something other than itself)
 * live in the test suite: brute-force longest paths on every small pattern,
 * lattice closed forms for grid Laplacians, dense linear algebra for the
 * rewrite, SciPy for the solve, finite differences for the adjoint,
 * hand-worked cases for the generator and the environment step (whose
 * reward constants and abandonment penalty are readings, stated there), a
 * plain-Python second implementation of the environment.  The
 * choice of the population standard deviation in the CV (see below) is a
 * definition the paper does not fix: parity unpinned on that one point.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status codes (same meanings as the GPU library's, independent numbering
 * is not needed: the tests compare meanings through these constants) */
enum {
    ORC_OK = 0,
    ORC_INVALID_ARG = -1,
    ORC_NOT_LOWER = -2,
    ORC_UNSORTED_OR_DUP = -3,
    ORC_MISSING_DIAG = -4,
    ORC_ZERO_DIAG = -5,
    ORC_BAD_ROWSET = -6,
    ORC_BUFFER_TOO_SMALL = -7,
};

/* ------------------------------------------------------------------------
 * validate: the CSR must describe a lower-triangular matrix with a stored,
 * nonzero diagonal (Section 2.1: L is lower triangular, each unknown needs
 * its own diagonal entry).  The reported error is the one of the lowest
 * offending row; inside that row the first offending entry decides, an
 * entry above the diagonal beating an out-of-order entry.  A row whose
 * entries are fine but whose last entry is not the diagonal reports
 * MISSING_DIAG; a stored diagonal equal to zero reports ZERO_DIAG (only
 * checked when values are given).  *bad_row receives the row (or -1).
 * ---------------------------------------------------------------------- */
int orc_validate(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                 const double *vals, int32_t *bad_row)
{
    *bad_row = -1;
    if (n < 0 || rowptr[0] != 0)
        return ORC_INVALID_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return ORC_INVALID_ARG;
    for (int32_t i = 0; i < n; ++i) {
        int32_t b = rowptr[i], e = rowptr[i + 1];
        for (int32_t p = b; p < e; ++p) {
            int32_t c = colidx[p];
            if (c < 0 || c > i) { *bad_row = i; return ORC_NOT_LOWER; }
            if (p > b && c <= colidx[p - 1]) { *bad_row = i; return ORC_UNSORTED_OR_DUP; }
        }
        if (e == b || colidx[e - 1] != i) { *bad_row = i; return ORC_MISSING_DIAG; }
        if (vals && vals[e - 1] == 0.0) { *bad_row = i; return ORC_ZERO_DIAG; }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Exact unsigned 128-bit integers for the CV numerator.
 * ---------------------------------------------------------------------- */
typedef unsigned __int128 u128;

/* CV of a list of nonnegative integers a[0..D-1] (Section 4.1 and the
 * features of Table 1): sqrt(D*S2 - S1^2) / S1 with S1 = sum a, S2 = sum a^2.
 * This is the population standard deviation over the mean, written so that
 * everything before the square root is exact: the numerator is formed in
 * 128-bit integers, converted to double once (round to nearest), then one
 * IEEE sqrt and one IEEE divide.  D == 1 or S1 == 0 gives 0. */
static double cv_of(const int64_t *a, int32_t D, uint64_t *S1_out, u128 *S2_out)
{
    uint64_t S1 = 0;
    u128 S2 = 0;
    for (int32_t l = 0; l < D; ++l) {
        S1 += (uint64_t)a[l];
        S2 += (u128)(uint64_t)a[l] * (u128)(uint64_t)a[l];
    }
    if (S1_out) *S1_out = S1;
    if (S2_out) *S2_out = S2;
    if (D <= 1 || S1 == 0)
        return 0.0;
    u128 num = (u128)(uint64_t)D * S2 - (u128)S1 * (u128)S1;
    return sqrt((double)num) / (double)S1;
}

typedef struct {
    int32_t num_levels;     /* D */
    int32_t thin_count;     /* levels with cost < thin threshold */
    uint64_t S1;            /* sum of level costs */
    uint64_t S2_lo, S2_hi;  /* sum of squared level costs, 128-bit */
    double cv;              /* CV of level costs */
    double cv_rows;         /* CV of rows per level */
    double alc;             /* average level cost  S1 / D */
    double arl;             /* average rows per level  n / D */
    double air;             /* average incoming dependencies per row */
    double thin_threshold;  /* ALC * (1 + max(0, 1 - CV)) */
} orc_stats;

/* ------------------------------------------------------------------------
 * analyze (Section 2.1, level-set method; Section 4.1, environment features)
 *
 * level[i] = 0 when row i has no off-diagonal entry, otherwise
 * 1 + max level over its off-diagonal columns: the longest dependency path
 * ending at row i.  Because every dependency of row i has a smaller index,
 * visiting rows in index order is a topological order.
 *
 * rows[l]  = number of rows on level l,
 * cost[l]  = sum over rows on level l of (2*nnz_i - 1), nnz_i counting the
 *            diagonal: one multiply and one subtract per dependency plus the
 *            division by the diagonal.  (The paper does not spell out the row
 *            cost; this one reproduces its printed ALC = (2 nnz - n)/levels
 *            for all eight matrices of Tables 2, 4 and 5.)
 * perm     = rows ordered by (level, row index); level_ptr = offsets of the
 *            levels in perm.
 * Capacities: level[n], rows[n], cost[n], perm[n], level_ptr[n+1].
 * Returns D (> 0) or 0 for n == 0.
 * ---------------------------------------------------------------------- */
int32_t orc_analyze(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                    int32_t *level, int32_t *rows, int64_t *cost,
                    int32_t *perm, int32_t *level_ptr, orc_stats *st)
{
    memset(st, 0, sizeof *st);
    if (n == 0) { level_ptr[0] = 0; return 0; }
    int32_t D = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t lv = 0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1] - 1; ++p) {
            int32_t j = colidx[p];
            if (level[j] + 1 > lv) lv = level[j] + 1;
        }
        level[i] = lv;
        if (lv + 1 > D) D = lv + 1;
    }
    for (int32_t l = 0; l < D; ++l) { rows[l] = 0; cost[l] = 0; }
    for (int32_t i = 0; i < n; ++i) {
        int64_t nnz_i = rowptr[i + 1] - rowptr[i];
        rows[level[i]] += 1;
        cost[level[i]] += 2 * nnz_i - 1;
    }
    /* counting sort by level, stable in row order */
    level_ptr[0] = 0;
    for (int32_t l = 0; l < D; ++l) level_ptr[l + 1] = level_ptr[l] + rows[l];
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    for (int32_t l = 0; l < D; ++l) cur[l] = level_ptr[l];
    for (int32_t i = 0; i < n; ++i) perm[cur[level[i]]++] = i;
    free(cur);

    u128 S2;
    uint64_t S1;
    st->num_levels = D;
    st->cv = cv_of(cost, D, &S1, &S2);
    st->S1 = S1;
    st->S2_lo = (uint64_t)S2;
    st->S2_hi = (uint64_t)(S2 >> 64);
    int64_t *r64 = (int64_t *)malloc(sizeof(int64_t) * (size_t)D);
    for (int32_t l = 0; l < D; ++l) r64[l] = rows[l];
    st->cv_rows = cv_of(r64, D, NULL, NULL);
    free(r64);
    int64_t nnz = rowptr[n];
    st->alc = (double)S1 / (double)D;
    st->arl = (double)n / (double)D;
    st->air = (double)(nnz - n) / (double)n;
    /* relaxed thin-level threshold of Section 4.1 with alpha = 1 */
    double relax = 1.0 - st->cv;
    if (relax < 0.0) relax = 0.0;
    st->thin_threshold = st->alc * (1.0 + 1.0 * relax);
    int32_t thin = 0;
    for (int32_t l = 0; l < D; ++l)
        if ((double)cost[l] < st->thin_threshold) ++thin;
    st->thin_count = thin;
    return D;
}

/* ------------------------------------------------------------------------
 * Equation rewriting (Section 2.2): a rewritten row r with target level t
 * replaces each of its dependencies j that sits on level >= t by row j's
 * own equation, i.e. subtracts c * (row j of L) with c chosen to cancel the
 * entry at column j, and does the same to the right-hand side.  Newly
 * introduced dependencies at level >= t are substituted in turn, always
 * taking the largest such column first, until every remaining dependency
 * sits below the target.  The substituted rows are the *input* rows, so a
 * row set is applied all at once against L.  Entries that cancel to zero
 * numerically stay in the pattern.  Rows not in the set are copied.
 *
 * Row set: rows[0..m-1] strictly ascending; targets[q] the target level of
 * rows[q] (NULL: level - 1).  A target >= the row's level, or a row on
 * level 0, leaves the row unchanged.  A negative target is an error.
 *
 * Output (caller allocates, capacities checked):
 *   out_rowptr[n+1], out_colidx/out_vals[cap_nnz]: L' in CSR;
 *   Bp (n x k, ldbp): B' = M B, where M = I - C;
 *   C in CSR over the m set rows: c_ptr[m+1], c_col/c_val[cap_c], one
 *   (column j, multiplier c) per substitution, in substitution order.
 * sizes[0] = nnz(L'), sizes[1] = nnz(C), sizes[2] = rows left unchanged.
 * With cap_nnz or cap_c too small only sizes are filled and
 * ORC_BUFFER_TOO_SMALL is returned.
 * ---------------------------------------------------------------------- */

/* sparse accumulator: dense value array + membership flags + list */
typedef struct {
    double *val;
    unsigned char *in;
    int32_t *list;
    int32_t len;
} spa_t;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int orc_rewrite(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                const double *vals, const int32_t *level,
                int32_t m, const int32_t *set_rows, const int32_t *targets,
                int32_t k, const double *B, int64_t ldb,
                int32_t *out_rowptr, int32_t *out_colidx, double *out_vals,
                int64_t cap_nnz, double *Bp, int64_t ldbp,
                int32_t *c_ptr, int32_t *c_col, double *c_val, int64_t cap_c,
                int64_t *sizes)
{
    for (int32_t q = 0; q < m; ++q) {
        if (set_rows[q] < 0 || set_rows[q] >= n) return ORC_BAD_ROWSET;
        if (q > 0 && set_rows[q] <= set_rows[q - 1]) return ORC_BAD_ROWSET;
        if (targets && targets[q] < 0) return ORC_BAD_ROWSET;
    }
    spa_t acc;
    acc.val = (double *)calloc((size_t)n, sizeof(double));
    acc.in = (unsigned char *)calloc((size_t)n, 1);
    acc.list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    double *rhs = (double *)malloc(sizeof(double) * (size_t)(k ? k : 1));
    int fits = 1;
    int64_t nnz_out = 0, nnz_c = 0, skipped = 0;
    int32_t q = 0;
    if (out_rowptr) out_rowptr[0] = 0;
    if (c_ptr) c_ptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int in_set = (q < m && set_rows[q] == i);
        int32_t t = -1;
        if (in_set) t = targets ? targets[q] : level[i] - 1;
        if (!in_set || level[i] == 0 || t >= level[i]) {
            /* copy row i and its right-hand side unchanged */
            if (in_set) ++skipped;
            int64_t len = rowptr[i + 1] - rowptr[i];
            if (fits && nnz_out + len <= cap_nnz && out_colidx) {
                memcpy(out_colidx + nnz_out, colidx + rowptr[i], sizeof(int32_t) * (size_t)len);
                memcpy(out_vals + nnz_out, vals + rowptr[i], sizeof(double) * (size_t)len);
            } else fits = 0;
            nnz_out += len;
            if (Bp)
                for (int32_t c = 0; c < k; ++c) Bp[i + c * ldbp] = B[i + c * ldb];
            if (out_rowptr) out_rowptr[i + 1] = (int32_t)nnz_out;
            if (in_set) { if (c_ptr) c_ptr[q + 1] = (int32_t)nnz_c; ++q; }
            continue;
        }
        /* load row i into the accumulator */
        acc.len = 0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t c = colidx[p];
            acc.val[c] = vals[p];
            acc.in[c] = 1;
            acc.list[acc.len++] = c;
        }
        for (int32_t c = 0; c < k; ++c) rhs[c] = B[i + c * ldb];
        for (;;) {
            /* largest column j != i still present with level[j] >= t */
            int32_t j = -1;
            for (int32_t s = 0; s < acc.len; ++s) {
                int32_t c = acc.list[s];
                if (c != i && acc.in[c] && level[c] >= t && c > j) j = c;
            }
            if (j < 0) break;
            double djj = vals[rowptr[j + 1] - 1];
            double cmul = acc.val[j] / djj;
            acc.in[j] = 0;
            acc.val[j] = 0.0;
            if (fits && nnz_c < cap_c && c_col) { c_col[nnz_c] = j; c_val[nnz_c] = cmul; }
            else fits = 0;
            ++nnz_c;
            for (int32_t p = rowptr[j]; p < rowptr[j + 1] - 1; ++p) {
                int32_t c = colidx[p];
                double prod = cmul * vals[p];
                if (acc.in[c]) {
                    acc.val[c] = acc.val[c] - prod;
                } else {
                    /* a column eliminated earlier cannot come back: every
                     * later substitution is of a smaller row, whose columns
                     * are all smaller than it */
                    acc.in[c] = 1;
                    acc.val[c] = 0.0 - prod;
                    acc.list[acc.len++] = c;
                }
            }
            for (int32_t c = 0; c < k; ++c) {
                double prod = cmul * B[j + c * ldb];
                rhs[c] = rhs[c] - prod;
            }
        }
        /* emit the surviving entries in ascending column order */
        int32_t live = 0;
        for (int32_t s = 0; s < acc.len; ++s)
            if (acc.in[acc.list[s]]) acc.list[live++] = acc.list[s];
        acc.len = live;
        qsort(acc.list, (size_t)live, sizeof(int32_t), cmp_i32);
        if (fits && nnz_out + live <= cap_nnz && out_colidx) {
            for (int32_t s = 0; s < live; ++s) {
                out_colidx[nnz_out + s] = acc.list[s];
                out_vals[nnz_out + s] = acc.val[acc.list[s]];
            }
        } else fits = 0;
        nnz_out += live;
        for (int32_t s = 0; s < live; ++s) { acc.in[acc.list[s]] = 0; acc.val[acc.list[s]] = 0.0; }
        if (Bp)
            for (int32_t c = 0; c < k; ++c) Bp[i + c * ldbp] = rhs[c];
        if (out_rowptr) out_rowptr[i + 1] = (int32_t)nnz_out;
        if (c_ptr) c_ptr[q + 1] = (int32_t)nnz_c;
        ++q;
    }
    free(acc.val); free(acc.in); free(acc.list); free(rhs);
    sizes[0] = nnz_out;
    sizes[1] = nnz_c;
    sizes[2] = skipped;
    if (nnz_out > cap_nnz || nnz_c > cap_c || !fits)
        return ORC_BUFFER_TOO_SMALL;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * solve: forward substitution L X = B (Section 2.1).  For i ascending and
 * each right-hand side: s = b_i, s -= L_ij x_j over the off-diagonal
 * entries in ascending column order, x_i = s / L_ii.
 * ---------------------------------------------------------------------- */
void orc_solve(int32_t n, const int32_t *rowptr, const int32_t *colidx,
               const double *vals, int32_t k, const double *B, int64_t ldb,
               double *X, int64_t ldx)
{
    for (int32_t c = 0; c < k; ++c) {
        const double *b = B + c * ldb;
        double *x = X + c * ldx;
        for (int32_t i = 0; i < n; ++i) {
            double s = b[i];
            int32_t e = rowptr[i + 1] - 1;
            for (int32_t p = rowptr[i]; p < e; ++p) {
                double prod = vals[p] * x[colidx[p]];
                s = s - prod;
            }
            x[i] = s / vals[e];
        }
    }
}

/* ------------------------------------------------------------------------
 * solve_upper: backward substitution U X = B for an upper-triangular CSR U
 * whose rows hold the diagonal first, then ascending columns (the U factor
 * of an incomplete LU, applied after L in a preconditioned iteration).  For
 * i descending and each right-hand side: s = b_i, s -= U_ij x_j over the
 * off-diagonal entries in ascending column order, x_i = s / U_ii.
 * ---------------------------------------------------------------------- */
void orc_solve_upper(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                     const double *vals, int32_t k, const double *B, int64_t ldb,
                     double *X, int64_t ldx)
{
    for (int32_t c = 0; c < k; ++c) {
        const double *b = B + c * ldb;
        double *x = X + c * ldx;
        for (int32_t i = n - 1; i >= 0; --i) {
            double s = b[i];
            int32_t d = rowptr[i];
            for (int32_t p = d + 1; p < rowptr[i + 1]; ++p) {
                double prod = vals[p] * x[colidx[p]];
                s = s - prod;
            }
            x[i] = s / vals[d];
        }
    }
}

/* ------------------------------------------------------------------------
 * Adjoint of x = L^{-1} b.  With y = L^{-T} g (backward substitution on the
 * transposed system) the gradients are grad_b = y and
 * grad_L[i][j] = -y_i x_j, summed over right-hand sides, on L's stored
 * pattern (diagonal included).
 *
 * solve_transpose: r = G; for i descending: y_i = r_i / L_ii, then for every
 * off-diagonal (j, v) of row i: r_j -= v * y_i.
 * ---------------------------------------------------------------------- */
void orc_solve_transpose(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                         const double *vals, int32_t k, const double *G, int64_t ldg,
                         double *Y, int64_t ldy)
{
    for (int32_t c = 0; c < k; ++c) {
        double *y = Y + c * ldy;
        for (int32_t i = 0; i < n; ++i) y[i] = G[i + c * ldg];
        for (int32_t i = n - 1; i >= 0; --i) {
            int32_t e = rowptr[i + 1] - 1;
            double yi = y[i] / vals[e];
            y[i] = yi;
            for (int32_t p = rowptr[i]; p < e; ++p) {
                double prod = vals[p] * yi;
                y[colidx[p]] = y[colidx[p]] - prod;
            }
        }
    }
}

void orc_grad_vals(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                   int32_t k, const double *Y, int64_t ldy, const double *X,
                   int64_t ldx, double *gvals)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double s = 0.0;
            for (int32_t c = 0; c < k; ++c) {
                double prod = Y[i + c * ldy] * X[colidx[p] + c * ldx];
                s = s + prod;
            }
            gvals[p] = 0.0 - s;
        }
}

/* ------------------------------------------------------------------------
 * Rewrite-list generator: the environment of Section 4.1 driven by a fixed
 * policy instead of the learned one, with the node choice of Section 4.3
 * and the target selection of Algorithm 1.  Written as plain scans over
 * the level table at every step.
 *
 * State (Section 4.1, updated after each move without touching the DAG):
 * the level of every row, and per level its cost (sum of 2*nnz_i - 1 over
 * its rows, the row keeping its original cost when it moves), its row count
 * and its indegree (sum of the dependency counts nnz_i - 1 of its rows).
 * Level numbers never change; a level whose last row leaves is empty
 * (collapsed) and is skipped by every search.
 *
 * thr = ALC * (1 + alpha * max(0, 1 - CV)) with the ALC and CV of the
 * input (Section 4.1), fixed for the whole run; a level is thin when it is
 * non-empty and its cost < thr.  T0 = thin levels at the start.
 *
 * One step:
 *   source: among levels l >= 1 that are thin, never a target and not
 *     rejected, the one with the fewest rows, ties to the lower level (a
 *     level keeps being chosen until it empties: its row count only falls);
 *   node: among the source's rows, the one with the fewest dependencies,
 *     ties to the lower row index (Section 4.3);
 *   target (Algorithm 1): p = nearest non-empty level above the source.
 *     p == 0: the target is level 0 when level 0 is thin, else the step
 *     is rejected.  p > 0: the target is the nearest thin level at or above
 *     p (all target affinities equal: the closest of the search window);
 *     with none, the fallback is p itself (a thin source may go to a thick
 *     level).  A target farther than max_dist levels rejects the step;
 *   a rejected step marks the source rejected (no later state change can
 *     make it acceptable: levels above a source only gain cost or empty);
 *   a move puts the node on the target level, updates the three per-level
 *     sums of source and target, marks the target as a target level, and
 *     appends <node, source, target> to the list.
 * Before each step, in this order: stop THIN when T0 > 0 and
 * thin / T0 < thin_stop; stop MOVES when the move limit (max_moves, 0 =
 * cap, never above cap) is reached; stop STEPS when max_steps steps (0 =
 * max(2 D, 3 * 2048)) were taken; stop NO_SOURCE when no source is left.
 *
 * Outputs: mv_row/mv_src/mv_tgt[cap] in move order; res (final non-empty
 * levels, thin levels, and S1, exact S2 and CV of the non-empty levels'
 * costs); out_cost/out_rows/out_deps[D] the final per-level sums (each
 * nullable).
 * ---------------------------------------------------------------------- */
enum { ORC_GEN_NO_SOURCE = 0, ORC_GEN_THIN = 1, ORC_GEN_MOVES = 2, ORC_GEN_STEPS = 3 };

typedef struct {
    double alpha;
    double thin_stop;
    int32_t max_dist;
    int32_t max_moves;
    int32_t max_steps;
    int32_t pad_;
} orc_gen_params;

typedef struct {
    int32_t moves, steps, stop, levels, thin, thin0, rejected, pad_;
    double threshold;
    uint64_t S1, S2_lo, S2_hi;
    double cv;
} orc_gen_result;

int orc_generate(int32_t n, const int32_t *rowptr, const int32_t *level, int32_t D,
                 double alc, double cv, const orc_gen_params *prm, int32_t cap,
                 int32_t *mv_row, int32_t *mv_src, int32_t *mv_tgt, orc_gen_result *res,
                 int64_t *out_cost, int32_t *out_rows, int64_t *out_deps)
{
    memset(res, 0, sizeof *res);
    if (n < 0 || D < 0 || cap < 0 || prm->max_dist < 0 || prm->max_moves < 0 ||
        prm->max_steps < 0 || !(prm->alpha >= 0.0) || !(prm->thin_stop >= 0.0) ||
        (n > 0 && D < 1))
        return ORC_INVALID_ARG;
    if (n == 0) return ORC_OK;

    int32_t *lev = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *cost = (int64_t *)calloc((size_t)D, sizeof(int64_t));
    int64_t *deps = (int64_t *)calloc((size_t)D, sizeof(int64_t));
    int32_t *rows = (int32_t *)calloc((size_t)D, sizeof(int32_t));
    unsigned char *is_target = (unsigned char *)calloc((size_t)D, 1);
    unsigned char *rejected = (unsigned char *)calloc((size_t)D, 1);
    /* rows of each original level, ascending (counting sort) */
    int32_t *optr = (int32_t *)calloc((size_t)D + 1, sizeof(int32_t));
    int32_t *orows = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) optr[level[i] + 1] += 1;
    for (int32_t l = 0; l < D; ++l) optr[l + 1] += optr[l];
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    for (int32_t l = 0; l < D; ++l) cur[l] = optr[l];
    for (int32_t i = 0; i < n; ++i) orows[cur[level[i]]++] = i;
    free(cur);
    for (int32_t i = 0; i < n; ++i) {
        int64_t d = rowptr[i + 1] - rowptr[i] - 1;
        lev[i] = level[i];
        cost[lev[i]] += 2 * d + 1;
        deps[lev[i]] += d;
        rows[lev[i]] += 1;
    }
    double relax = 1.0 - cv;
    if (relax < 0.0) relax = 0.0;
    double scaled = prm->alpha * relax;
    double factor = 1.0 + scaled;
    const double thr = alc * factor;
#define THIN(l) (rows[(l)] > 0 && (double)cost[(l)] < thr)
    int32_t T0 = 0;
    for (int32_t l = 0; l < D; ++l) T0 += THIN(l) ? 1 : 0;
    int32_t max_moves = prm->max_moves > 0 && prm->max_moves < cap ? prm->max_moves : cap;
    int64_t steps_default = 2 * (int64_t)D < 6144 ? 6144 : 2 * (int64_t)D;
    if (steps_default > INT32_MAX) steps_default = INT32_MAX;
    int32_t max_steps = prm->max_steps > 0 ? prm->max_steps : (int32_t)steps_default;
    int32_t moves = 0, steps = 0, nrej = 0, stop;

    for (;;) {
        int32_t thin = 0;
        for (int32_t l = 0; l < D; ++l) thin += THIN(l) ? 1 : 0;
        if (T0 > 0 && (double)thin / (double)T0 < prm->thin_stop) { stop = ORC_GEN_THIN; break; }
        if (moves >= max_moves) { stop = ORC_GEN_MOVES; break; }
        if (steps >= max_steps) { stop = ORC_GEN_STEPS; break; }
        int32_t src = -1;
        for (int32_t l = 1; l < D; ++l) {
            if (!THIN(l) || is_target[l] || rejected[l]) continue;
            if (src < 0 || rows[l] < rows[src]) src = l;
        }
        if (src < 0) { stop = ORC_GEN_NO_SOURCE; break; }
        steps += 1;

        /* a source never received rows (it is not a target), so its rows
         * are the unmoved ones among its original rows */
        int32_t node = -1;
        int64_t node_deps = 0;
        for (int32_t q = optr[src]; q < optr[src + 1]; ++q) {
            int32_t i = orows[q];
            if (lev[i] != src) continue;
            int64_t d = rowptr[i + 1] - rowptr[i] - 1;
            if (node < 0 || d < node_deps) { node = i; node_deps = d; }
        }

        int32_t p = src - 1;
        while (p > 0 && rows[p] == 0) --p;
        int32_t tgt;
        if (p == 0) {
            tgt = THIN(0) ? 0 : -1;
        } else {
            tgt = -1;
            for (int32_t l = p; l >= 0; --l)
                if (THIN(l)) { tgt = l; break; }
            if (tgt < 0) tgt = p;
        }
        if (tgt >= 0 && src - tgt > prm->max_dist) tgt = -1;
        if (tgt < 0) {
            rejected[src] = 1;
            nrej += 1;
            continue;
        }

        lev[node] = tgt;
        cost[src] -= 2 * node_deps + 1;
        deps[src] -= node_deps;
        rows[src] -= 1;
        cost[tgt] += 2 * node_deps + 1;
        deps[tgt] += node_deps;
        rows[tgt] += 1;
        is_target[tgt] = 1;
        mv_row[moves] = node;
        mv_src[moves] = src;
        mv_tgt[moves] = tgt;
        moves += 1;
    }

    int32_t nonempty = 0, thin = 0;
    int64_t *ne = (int64_t *)malloc(sizeof(int64_t) * (size_t)D);
    for (int32_t l = 0; l < D; ++l) {
        if (rows[l] > 0) ne[nonempty++] = cost[l];
        thin += THIN(l) ? 1 : 0;
    }
#undef THIN
    u128 S2;
    uint64_t S1;
    res->cv = cv_of(ne, nonempty, &S1, &S2);
    res->S1 = S1;
    res->S2_lo = (uint64_t)S2;
    res->S2_hi = (uint64_t)(S2 >> 64);
    res->moves = moves;
    res->steps = steps;
    res->stop = stop;
    res->levels = nonempty;
    res->thin = thin;
    res->thin0 = T0;
    res->rejected = nrej;
    res->threshold = thr;
    for (int32_t l = 0; l < D; ++l) {
        if (out_cost) out_cost[l] = cost[l];
        if (out_rows) out_rows[l] = rows[l];
        if (out_deps) out_deps[l] = deps[l];
    }
    free(ne);
    free(optr);
    free(orows);
    free(lev);
    free(cost);
    free(deps);
    free(rows);
    free(is_target);
    free(rejected);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Environment step with the reward of Algorithm 2 (Sections 4.1-4.5).
 *
 * One environment over the level table of L, driven from outside: each step
 * takes an action (a source level) and returns the reward.  State
 * (Section 4.1, the DAG is never modified): the level of every row, and
 * per level its cost, row count and dependency sum (a moved row keeps its
 * original cost 2*nnz_i - 1 and dependency count nnz_i - 1); per level also
 * whether it ever received a row, its initial size and first-touch step
 * (abandonment, Section 4.4), and the steps at which it was last chosen as
 * source and last received a row (the affinities of Section 4.2).
 *
 * Readings (the paper leaves these open; stated here and pinned by
 * hand-worked cases):
 *  - thr = ALC * (1 + alpha * max(0, 1 - CV)) of the input, fixed; thin =
 *    non-empty and cost < thr; levels, CV = over the non-empty levels.
 *  - action a is valid when 1 <= a < D and level a is non-empty; the mask
 *    heuristics of Section 4.3 shape the mask given to the policy
 *    (env_observe) and do not change validity.  An invalid action, or one
 *    Algorithm 1 rejects, changes nothing but the step count and earns
 *    -reward_alpha.
 *  - node: the row of level a with the fewest dependencies, ties to the
 *    lower row index (Section 4.3); rows that moved in may move again.
 *  - Algorithm 1: p = nearest non-empty level above a.  p == 0: target 0
 *    when level 0 is thin, else reject.  p > 0: among the search_window
 *    nearest thin levels at or above p, the one with the highest target
 *    affinity (the one that most recently received a row; never = lowest;
 *    ties to the nearest); with no thin level at or above p the fallback is
 *    p when the source is thin, else reject.  Reject when a - t > max_dist.
 *  - affinity of a level (observation): decay^(steps - stamp) with the step
 *    stamp of the last choice as source / last received row, 0 if never,
 *    -1 when the level is empty or, for the source affinity, ever received
 *    a row, or, for the target affinity, is not thin.  Comparisons of
 *    affinities are comparisons of stamps, exact.
 *  - reward of a move (Algorithm 2), dCV = CV before - CV after:
 *      r_cv = -reward_alpha if dCV < -eps; D0 * dCV if dCV > eps; else 0
 *      s = log(1 + size + 1), size = source rows before the move
 *      r_cp = reward_alpha * (D0 / levels after) * (1 + 1/s) if the source
 *             emptied; reward_alpha / s if the source was thin; else
 *             -reward_alpha * (1 + s)
 *      r_rwdist = log1p(thd - d) / D0 if d < thd, else -log1p(d - thd) / D0,
 *             d = a - t, thd = dist_threshold
 *      r_abandon (A = the previous move's source, when A != a): if A ever
 *             received a row, its initial size becomes its current size and
 *             its first touch 0, no penalty; no penalty when A is empty, or
 *             when a level >= 1 with exactly one row exists and A is thin;
 *             else -(1 - c) * log1p(step - first touch of A), with the
 *             completion ratio c = 1 - rows/(initial size + 1)
 *      reward = 0.80 r_cv + 0.80 r_cp + 0.05 r_rwdist + 0.50 r_abandon.
 *  - the episode ends (checked after reset and after each step, in this
 *    order): THIN when T0 > 0 and thin / T0 < thin_stop; MOVES when cap
 *    moves were made; STEPS when max_steps steps were taken (0 = max(2 D,
 *    6144)); NO_SOURCE when no level >= 1 is non-empty.  Later actions are
 *    ignored (reward 0) until reset.
 * ---------------------------------------------------------------------- */
typedef struct {
    double alpha;
    double thin_stop;
    double reward_alpha;
    double eps;
    double decay;
    int32_t max_dist;
    int32_t search_window;
    int32_t dist_threshold;
    int32_t max_steps;
    int32_t stall_steps;
    int32_t keep_top;
} orc_env_params;

enum { ORC_ENV_MOVED = 0, ORC_ENV_INVALID = 1, ORC_ENV_REJECTED = 2, ORC_ENV_IGNORED = 3 };

typedef struct {
    int32_t outcome, node, src, tgt, collapsed, done;
    int32_t steps, moves, levels, thin, thin0, pad_;
    double reward, r_cv, r_cp, r_rwdist, r_abandon, cv, cv_rows;
} orc_env_result;

typedef struct {
    int32_t n, D, cap;
    orc_env_params prm;
    double thr, alc, arl;
    int32_t *deps_row;   /* nnz_i - 1 */
    const int32_t *level0;
    int32_t *lev;
    int64_t *cost, *deps;
    int32_t *rows, *init_size, *first, *sstamp, *tstamp;
    unsigned char *is_target;
    int32_t steps, moves, last_src, last_collapse, T0, D0, done, max_steps;
    int32_t *mv_row, *mv_src, *mv_tgt;
} orc_env;

static int env_thin(const orc_env *v, int32_t l)
{
    return v->rows[l] > 0 && (double)v->cost[l] < v->thr;
}

static int32_t env_count_thin(const orc_env *v)
{
    int32_t t = 0;
    for (int32_t l = 0; l < v->D; ++l) t += env_thin(v, l);
    return t;
}

static int32_t env_levels(const orc_env *v)
{
    int32_t t = 0;
    for (int32_t l = 0; l < v->D; ++l) t += v->rows[l] > 0;
    return t;
}

/* CV of the non-empty levels' costs and of their row counts */
static void env_cvs(const orc_env *v, double *cv_cost, double *cv_rows)
{
    int64_t *a = (int64_t *)malloc(sizeof(int64_t) * (size_t)v->D);
    int64_t *b = (int64_t *)malloc(sizeof(int64_t) * (size_t)v->D);
    int32_t m = 0;
    for (int32_t l = 0; l < v->D; ++l)
        if (v->rows[l] > 0) {
            a[m] = v->cost[l];
            b[m] = v->rows[l];
            ++m;
        }
    *cv_cost = cv_of(a, m, NULL, NULL);
    *cv_rows = cv_of(b, m, NULL, NULL);
    free(a);
    free(b);
}

static int32_t env_stop(const orc_env *v)
{
    int32_t thin = env_count_thin(v);
    if (v->T0 > 0 && (double)thin / (double)v->T0 < v->prm.thin_stop) return ORC_GEN_THIN;
    if (v->moves >= v->cap) return ORC_GEN_MOVES;
    if (v->steps >= v->max_steps) return ORC_GEN_STEPS;
    int32_t any = 0;
    for (int32_t l = 1; l < v->D; ++l) any |= v->rows[l] > 0;
    if (!any) return ORC_GEN_NO_SOURCE;
    return -1;
}

void orc_env_reset(orc_env *v)
{
    memset(v->cost, 0, sizeof(int64_t) * (size_t)v->D);
    memset(v->deps, 0, sizeof(int64_t) * (size_t)v->D);
    memset(v->rows, 0, sizeof(int32_t) * (size_t)v->D);
    for (int32_t i = 0; i < v->n; ++i) {
        int32_t l = v->level0[i];
        v->lev[i] = l;
        v->cost[l] += 2 * (int64_t)v->deps_row[i] + 1;
        v->deps[l] += v->deps_row[i];
        v->rows[l] += 1;
    }
    for (int32_t l = 0; l < v->D; ++l) {
        v->init_size[l] = v->rows[l];
        v->first[l] = 0;
        v->sstamp[l] = 0;
        v->tstamp[l] = 0;
        v->is_target[l] = 0;
    }
    v->steps = 0;
    v->moves = 0;
    v->last_src = -1;
    v->last_collapse = 0;
    v->T0 = env_count_thin(v);
    v->D0 = env_levels(v);
    v->done = env_stop(v);
}

void orc_env_destroy(orc_env *v)
{
    if (!v) return;
    free(v->deps_row);
    free(v->lev);
    free(v->cost);
    free(v->deps);
    free(v->rows);
    free(v->init_size);
    free(v->first);
    free(v->sstamp);
    free(v->tstamp);
    free(v->is_target);
    free(v->mv_row);
    free(v->mv_src);
    free(v->mv_tgt);
    free(v);
}

/* level: the analysis' level of every row (kept by pointer: the caller
 * keeps it alive while the environment exists).  Returns NULL on bad
 * arguments. */
orc_env *orc_env_create(int32_t n, const int32_t *rowptr, const int32_t *level, int32_t D,
                        double alc, double cv, const orc_env_params *prm, int32_t cap)
{
    if (n < 1 || D < 1 || D > n || cap < 0 || !(prm->alpha >= 0.0) || !(prm->thin_stop >= 0.0) ||
        !(prm->decay > 0.0 && prm->decay < 1.0) || !(prm->eps >= 0.0) || prm->max_dist < 0 ||
        prm->search_window < 1 || prm->max_steps < 0 || prm->stall_steps < 0 ||
        prm->keep_top < 1)
        return NULL;
    for (int32_t i = 0; i < n; ++i)
        if (level[i] < 0 || level[i] >= D) return NULL;
    orc_env *v = (orc_env *)calloc(1, sizeof(orc_env));
    v->n = n;
    v->D = D;
    v->cap = cap;
    v->prm = *prm;
    double relax = 1.0 - cv;
    if (relax < 0.0) relax = 0.0;
    double scaled = prm->alpha * relax;
    double factor = 1.0 + scaled;
    v->thr = alc * factor;
    v->alc = alc;
    v->arl = (double)n / (double)D;
    v->level0 = level;
    v->deps_row = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) v->deps_row[i] = rowptr[i + 1] - rowptr[i] - 1;
    v->lev = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    v->cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)D);
    v->deps = (int64_t *)malloc(sizeof(int64_t) * (size_t)D);
    v->rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    v->init_size = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    v->first = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    v->sstamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    v->tstamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    v->is_target = (unsigned char *)malloc((size_t)D);
    size_t cc = cap > 0 ? (size_t)cap : 1;
    v->mv_row = (int32_t *)malloc(sizeof(int32_t) * cc);
    v->mv_src = (int32_t *)malloc(sizeof(int32_t) * cc);
    v->mv_tgt = (int32_t *)malloc(sizeof(int32_t) * cc);
    int64_t ms = 2 * (int64_t)D < 6144 ? 6144 : 2 * (int64_t)D;
    if (ms > INT32_MAX) ms = INT32_MAX;
    v->max_steps = prm->max_steps > 0 ? prm->max_steps : (int32_t)ms;
    orc_env_reset(v);
    return v;
}

static void env_fill(const orc_env *v, orc_env_result *r)
{
    r->done = v->done;
    r->steps = v->steps;
    r->moves = v->moves;
    r->levels = env_levels(v);
    r->thin = env_count_thin(v);
    r->thin0 = v->T0;
    env_cvs(v, &r->cv, &r->cv_rows);
}

void orc_env_step(orc_env *v, int32_t a, orc_env_result *r)
{
    memset(r, 0, sizeof *r);
    r->node = r->src = r->tgt = -1;
    if (v->done >= 0) {
        r->outcome = ORC_ENV_IGNORED;
        env_fill(v, r);
        return;
    }
    const int32_t step = v->steps + 1;
    const double ra = v->prm.reward_alpha;
    int32_t t = -1, node = -1;
    int outcome = ORC_ENV_MOVED;
    if (a < 1 || a >= v->D || v->rows[a] == 0) {
        outcome = ORC_ENV_INVALID;
    } else {
        /* node: fewest dependencies, ties to the lower row */
        for (int32_t i = 0; i < v->n; ++i)
            if (v->lev[i] == a && (node < 0 || v->deps_row[i] < v->deps_row[node])) node = i;
        /* Algorithm 1 */
        int32_t p = a - 1;
        while (p > 0 && v->rows[p] == 0) --p;
        if (p == 0) {
            t = env_thin(v, 0) ? 0 : -1;
        } else {
            int32_t found = 0, best = -1;
            for (int32_t l = p; l >= 0 && found < v->prm.search_window; --l) {
                if (!env_thin(v, l)) continue;
                ++found;
                if (best < 0 || v->tstamp[l] > v->tstamp[best]) best = l;
            }
            if (best >= 0) t = best;
            else t = env_thin(v, a) ? p : -1;
        }
        if (t >= 0 && a - t > v->prm.max_dist) t = -1;
        if (t < 0) outcome = ORC_ENV_REJECTED;
    }
    v->steps = step;
    if (outcome != ORC_ENV_MOVED) {
        r->outcome = outcome;
        r->src = outcome == ORC_ENV_REJECTED ? a : -1;
        r->node = outcome == ORC_ENV_REJECTED ? node : -1;
        r->reward = -ra;
        v->done = env_stop(v);
        env_fill(v, r);
        return;
    }

    double cv_before, cvr_unused;
    env_cvs(v, &cv_before, &cvr_unused);
    const int32_t size = v->rows[a];
    const int src_thin = env_thin(v, a);

    /* abandonment of the previous source, on the state before the move */
    double r_ab = 0.0;
    const int32_t A = v->last_src;
    if (A >= 1 && A != a) {
        if (v->is_target[A]) {
            v->init_size[A] = v->rows[A];
            v->first[A] = 0;
        } else if (v->rows[A] > 0) {
            int32_t ones = 0;
            for (int32_t l = 1; l < v->D; ++l) ones += v->rows[l] == 1;
            if (!(ones > 0 && env_thin(v, A))) {
                double q = (double)v->rows[A] / ((double)v->init_size[A] + 1.0);
                double c = 1.0 - q;
                double pen = (1.0 - c) * log1p((double)(step - v->first[A]));
                r_ab = -pen;
            }
        }
    }

    /* the move */
    const int64_t d = v->deps_row[node];
    v->lev[node] = t;
    v->cost[a] -= 2 * d + 1;
    v->deps[a] -= d;
    v->rows[a] -= 1;
    v->cost[t] += 2 * d + 1;
    v->deps[t] += d;
    v->rows[t] += 1;
    v->is_target[t] = 1;
    v->tstamp[t] = step;
    v->sstamp[a] = step;
    if (v->first[a] == 0) v->first[a] = step;
    v->last_src = a;
    if (v->moves < v->cap) {
        v->mv_row[v->moves] = node;
        v->mv_src[v->moves] = a;
        v->mv_tgt[v->moves] = t;
    }
    v->moves += 1;
    const int collapsed = v->rows[a] == 0;
    if (collapsed) v->last_collapse = step;

    double cv_after, cvr_after;
    env_cvs(v, &cv_after, &cvr_after);
    const int32_t levels = env_levels(v);
    const double D0 = (double)v->D0;

    double dcv = cv_before - cv_after;
    double r_cv = 0.0;
    if (dcv < -v->prm.eps) r_cv = -ra;
    else if (dcv > v->prm.eps) r_cv = D0 * dcv;

    double s = log(1.0 + (double)size + 1.0);
    double r_cp;
    if (collapsed) r_cp = ra * (D0 / (double)levels) * (1.0 + 1.0 / s);
    else if (src_thin) r_cp = ra / s;
    else r_cp = -1.0 * ra * (1.0 + s);

    int32_t dist = a - t, thd = v->prm.dist_threshold;
    double r_rw;
    if (dist < thd) r_rw = log1p((double)(thd - dist)) / D0;
    else r_rw = -log1p((double)(dist - thd)) / D0;

    r->outcome = ORC_ENV_MOVED;
    r->node = node;
    r->src = a;
    r->tgt = t;
    r->collapsed = collapsed;
    r->r_cv = r_cv;
    r->r_cp = r_cp;
    r->r_rwdist = r_rw;
    r->r_abandon = r_ab;
    double w1 = 0.80 * r_cv;
    double w2 = 0.80 * r_cp;
    double w3 = 0.05 * r_rw;
    double w4 = 0.50 * r_ab;
    double sum = w1 + w2;
    sum = sum + w3;
    r->reward = sum + w4;
    v->done = env_stop(v);
    env_fill(v, r);
}

/* Observation of Section 4.2 (Table 1) and the action mask of Section 4.3.
 *   level[f * D + l], f = 0..5: cost / ALC, rows / ARL, source affinity,
 *     target affinity, completion ratio 1 - rows/(initial size + 1), thin
 *     (1 or 0); ALC and ARL of the input.
 *   global[9]: CV of level costs, 1 (its reference), CV of rows per level,
 *     1, levels / n, moves / n (rewrite ratio), thin / T0 (0 when T0 = 0),
 *     levels / D0 (critical-path ratio), thin / levels.
 *   mask[D]: 1 for a valid action (1 <= l, non-empty), all 0 once the
 *     episode ended; when the previous move's source has exactly one row
 *     left, only that level; otherwise, after stall_steps > 0 steps without
 *     a collapse, only the keep_top valid levels of highest source affinity
 *     (ties to the lower level; levels that received rows rank below
 *     untouched ones).
 * Each output is nullable. */
void orc_env_observe(const orc_env *v, double *level, double *global, unsigned char *mask)
{
    const int32_t D = v->D;
    const int32_t thin = env_count_thin(v), levels = env_levels(v);
    if (level) {
        for (int32_t l = 0; l < D; ++l) {
            int empty = v->rows[l] == 0;
            level[0 * D + l] = (double)v->cost[l] / v->alc;
            level[1 * D + l] = (double)v->rows[l] / v->arl;
            double sa, ta;
            if (empty || v->is_target[l]) sa = -1.0;
            else if (v->sstamp[l] == 0) sa = 0.0;
            else sa = pow(v->prm.decay, (double)(v->steps - v->sstamp[l]));
            if (!env_thin(v, l)) ta = -1.0;
            else if (v->tstamp[l] == 0) ta = 0.0;
            else ta = pow(v->prm.decay, (double)(v->steps - v->tstamp[l]));
            level[2 * D + l] = sa;
            level[3 * D + l] = ta;
            double q = (double)v->rows[l] / ((double)v->init_size[l] + 1.0);
            level[4 * D + l] = 1.0 - q;
            level[5 * D + l] = env_thin(v, l) ? 1.0 : 0.0;
        }
    }
    if (global) {
        double cvc, cvr;
        env_cvs(v, &cvc, &cvr);
        global[0] = cvc;
        global[1] = 1.0;
        global[2] = cvr;
        global[3] = 1.0;
        global[4] = (double)levels / (double)v->n;
        global[5] = (double)v->moves / (double)v->n;
        global[6] = v->T0 > 0 ? (double)thin / (double)v->T0 : 0.0;
        global[7] = (double)levels / (double)v->D0;
        global[8] = levels > 0 ? (double)thin / (double)levels : 0.0;
    }
    if (mask) {
        for (int32_t l = 0; l < D; ++l) mask[l] = v->done < 0 && l >= 1 && v->rows[l] > 0;
        if (v->done >= 0) return;
        if (v->last_src >= 1 && v->rows[v->last_src] == 1) {
            for (int32_t l = 0; l < D; ++l) mask[l] = l == v->last_src;
        } else if (v->prm.stall_steps > 0 && v->steps - v->last_collapse >= v->prm.stall_steps) {
            /* keep the keep_top best valid levels by (key desc, level asc) */
            unsigned char *keep = (unsigned char *)calloc((size_t)D, 1);
            for (int32_t k = 0; k < v->prm.keep_top; ++k) {
                int32_t best = -1;
                int64_t bkey = 0;
                for (int32_t l = 1; l < D; ++l) {
                    if (!mask[l] || keep[l]) continue;
                    int64_t key = v->is_target[l] ? -1 : v->sstamp[l];
                    if (best < 0 || key > bkey) { best = l; bkey = key; }
                }
                if (best < 0) break;
                keep[best] = 1;
            }
            for (int32_t l = 0; l < D; ++l) mask[l] = keep[l];
            free(keep);
        }
    }
}

/* State readout: current level of every row (nullable), per-level cost,
 * rows, dependency sums (each nullable), and the move list so far. */
void orc_env_state(const orc_env *v, int32_t *lev, int64_t *cost, int32_t *rows, int64_t *deps,
                   int32_t *mv_row, int32_t *mv_src, int32_t *mv_tgt)
{
    for (int32_t i = 0; lev && i < v->n; ++i) lev[i] = v->lev[i];
    for (int32_t l = 0; l < v->D; ++l) {
        if (cost) cost[l] = v->cost[l];
        if (rows) rows[l] = v->rows[l];
        if (deps) deps[l] = v->deps[l];
    }
    int32_t m = v->moves < v->cap ? v->moves : v->cap;
    for (int32_t q = 0; q < m; ++q) {
        if (mv_row) mv_row[q] = v->mv_row[q];
        if (mv_src) mv_src[q] = v->mv_src[q];
        if (mv_tgt) mv_tgt[q] = v->mv_tgt[q];
    }
}
