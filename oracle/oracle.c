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
 * rewrite, SciPy for the solve, finite differences for the adjoint.  The
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
 * policy instead of the learned one, with the node choice of Section 4.4
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
 *     ties to the lower row index (Section 4.4);
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
