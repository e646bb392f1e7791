/*
 * rwtrsv -- sparse triangular solve on equation-rewritten dependency DAGs,
 * with the level-set analysis that scores each rewrite.  MI355X (gfx950).
 *
 * The problem (paper Section 2.1): solve L X = B for a sparse lower
 * triangular L stored in CSR.  Row i is a node of a dependency DAG, each
 * off-diagonal entry L_ij an edge j -> i.  The level-set method groups rows
 * into levels (longest path from a source) that can be solved in parallel,
 * one level after another.  Equation rewriting (Section 2.2) replaces a
 * row's dependency on row j by row j's own equation, which moves the row to
 * an earlier level; the result is again a lower triangular CSR matrix L'
 * with a patched right-hand side B' and the same solution X.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Matrices: int32 rowptr[n+1], int32 colidx[nnz], values FP64 or FP32.
 *    Inside a row the columns strictly ascend and the diagonal is the last
 *    entry (rwt_validate checks this).  nnz < 2^31.
 *  - Dense blocks of k right-hand sides: column-major n x k, leading
 *    dimension ld >= n, same value type as the matrix.  An empty system
 *    (n = 0, or k = 0) is accepted by the solves, the adjoint calls and
 *    the upper-plan calls with NULL blocks, and does nothing; the empty
 *    matrix (rowptr = {0}, nnz = 0) may pass NULL colidx and values.
 *  - Every pointer argument named d_* (and every pointer inside rwt_csr) is
 *    device memory; h_* is host memory.  The library never allocates device
 *    memory: the caller passes a workspace of at least the size returned by
 *    the matching *_ws query and keeps it alive while a plan uses it.
 *  - Every call is ordered on the given HIP stream.  Calls that return
 *    host data (h_* outputs) synchronize that stream before returning.
 *  - Return value: RWT_OK or a negative rwt_status; rwt_last_error_string()
 *    (thread-local) describes the last failure of the calling thread.
 *    No call launches any kernel after detecting an argument error.
 */
#ifndef RWTRSV_H
#define RWTRSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* rwt_stream_t;   /* hipStream_t; NULL = default stream */

typedef enum {
    RWT_OK = 0,
    RWT_ERR_INVALID_ARG = -1,      /* null pointer, negative size, bad rowptr, ld < n */
    RWT_ERR_NOT_LOWER = -2,        /* an entry lies above the diagonal or col < 0 */
    RWT_ERR_UNSORTED_OR_DUP = -3,  /* columns of a row not strictly ascending */
    RWT_ERR_MISSING_DIAG = -4,     /* a row's last entry is not its diagonal */
    RWT_ERR_ZERO_DIAG = -5,        /* a stored diagonal equals zero */
    RWT_ERR_BAD_ROWSET = -6,       /* rewrite rows unsorted/duplicate/out of range, target < 0 */
    RWT_ERR_BUFFER_TOO_SMALL = -7, /* workspace or output capacity below what is needed */
    RWT_ERR_TOO_LARGE = -8,        /* sizes beyond the int32 index range or an internal limit */
    RWT_ERR_DEADLOCK = -9,         /* a bounded device wait expired (watchdog) */
    RWT_ERR_HIP = -10              /* HIP runtime error, see rwt_last_hip_error() */
} rwt_status;

typedef enum { RWT_F64 = 0, RWT_F32 = 1 } rwt_dtype;

/* A CSR view.  vals may be NULL for calls that use the pattern only. */
typedef struct {
    int32_t n;
    int32_t pad_;
    int64_t nnz;
    const int32_t* rowptr;   /* device, n+1 */
    const int32_t* colidx;   /* device, nnz */
    const void* vals;        /* device, nnz, type dt (nullable) */
    rwt_dtype dt;
    int32_t pad2_;
} rwt_csr;

/* Level statistics (Section 4.1 and Table 1: level count, per-level cost,
 * coefficient of variation of level costs and of level node counts, and
 * the ALC / ARL / AIR features of Section 3).
 * cost of a row = 2*nnz_row - 1 (one multiply and one subtract per
 * dependency and one division); S1 = sum of level costs = 2*nnz - n;
 * S2 = sum of squared level costs (exact, 128 bit);
 * cv = sqrt(D*S2 - S1^2)/S1 with the radicand exact before one rounding;
 * thin_threshold = ALC*(1 + max(0, 1 - cv)) (alpha = 1); thin_count =
 * number of levels with cost < thin_threshold. */
typedef struct {
    int32_t num_levels;
    int32_t thin_count;
    uint64_t S1;
    uint64_t S2_lo;
    uint64_t S2_hi;
    double cv;
    double cv_rows;
    double alc;
    double arl;
    double air;
    double thin_threshold;
    int32_t max_level_rows;   /* rows on the widest level */
    int32_t pad_;
} rwt_level_stats;

const char* rwt_last_error_string(void);
int rwt_last_hip_error(void);
/* "rwtrsv <major>.<minor> gfx950"; 0.2 added rwt_plan_opts.stage_outside
 * and rwt_plan_info.stage_outside (callers built against 0.1 must rebuild);
 * 0.3 added rwt_upper_levels, rwt_solve_withhold, rwt_batch_run_setup/_main,
 * rwt_source_hash and rwt_apply_M_noalloc */
const char* rwt_version(void);
/* 16 hex digits identifying the sources and flags the library was built
 * from ("unknown" when the build did not say) */
const char* rwt_source_hash(void);

/* ------------------------------------------------------------------------
 * Validation (CSR interchange format of Section 2.2).  Reports the error of
 * the lowest offending row (*h_bad_row, -1 when none or not row-specific);
 * inside the row the first offending entry decides, an entry above the
 * diagonal beating an out-of-order one; ZERO_DIAG is checked only when
 * L->vals is not NULL.  Workspace: rwt_validate_ws bytes.  Synchronizes.
 * ---------------------------------------------------------------------- */
size_t rwt_validate_ws(void);
rwt_status rwt_validate(const rwt_csr* L, void* d_ws, size_t ws_bytes,
                        int32_t* h_bad_row, rwt_stream_t stream);

/* ------------------------------------------------------------------------
 * Level-set analysis (Section 2.1: rows of one level are independent; the
 * level of row i is 0 without dependencies, else 1 + the largest level of
 * its dependencies).  Outputs (device, caller-allocated):
 *   d_level[n]        level of each row
 *   d_perm[n]         rows ordered by (level, row)
 *   d_level_ptr[n+1]  offsets of each level in d_perm (first D+1 used)
 *   d_rows[n]         rows per level (first D used)
 *   d_cost[n]         int64 cost per level (first D used)
 *   d_stats           statistics, device copy (always written)
 *   h_stats           host copy (nullable; non-NULL synchronizes)
 * Workspace: rwt_analyze_ws(L) bytes.  The pattern is assumed valid.
 * ---------------------------------------------------------------------- */
rwt_status rwt_analyze_ws(const rwt_csr* L, size_t* h_bytes);
rwt_status rwt_analyze(const rwt_csr* L, void* d_ws, size_t ws_bytes,
                       int32_t* d_level, int32_t* d_perm, int32_t* d_level_ptr,
                       int32_t* d_rows, int64_t* d_cost, rwt_level_stats* d_stats,
                       rwt_level_stats* h_stats, rwt_stream_t stream);

/* ------------------------------------------------------------------------
 * Equation rewriting (Section 2.2; the rewriting list of <node, source
 * level, target level> triplets of Algorithm 1).  For each rewritten row r
 * with target level t, every dependency j with level[j] >= t is replaced by
 * row j's equation: row r -= c*row j with c = (current entry at j)/L_jj,
 * and B'[r,:] -= c*B[j,:].  Substitutions introduced by this are applied in
 * turn, always taking the largest such column first, until every remaining
 * dependency lies below level t.  The substituted rows are those of the
 * input L (the whole set is applied at once).  Entries that cancel to zero
 * stay in the pattern.  Rows outside the set are copied.
 *
 * Row set: d_set_rows[m] strictly ascending, d_targets[m] (NULL: level-1).
 * A row on level 0 or with target >= its level is copied unchanged and
 * counted in sizes[2].  d_level must be the analysis of L.
 *
 * rwt_rewrite_symbolic computes d_rowptr_out[n+1] (L') and d_cptr_out[m+1]
 * (offsets of each set row's substitutions) and returns on the host
 * h_sizes[0] = nnz(L'), h_sizes[1] = number of substitutions,
 * h_sizes[2] = set rows left unchanged (synchronizes).
 * rwt_rewrite_numeric fills Lp->colidx/vals (capacity h_sizes[0]),
 * d_Bp (n x k, ldbp; may not alias d_B) and the multipliers:
 * d_crow/d_ccol/d_cval[h_sizes[1]]: substitution e subtracted
 * d_cval[e] * (row d_ccol[e]) from row d_crow[e]; so L' = M L and B' = M B
 * with M = I - C.  Multiplier arrays may be NULL.  Lp->rowptr must be the
 * d_rowptr_out of the symbolic call.  Workspace: rwt_rewrite_ws bytes
 * (same workspace, untouched in between, for both calls).
 * ---------------------------------------------------------------------- */
rwt_status rwt_rewrite_ws(const rwt_csr* L, int32_t m, size_t* h_bytes);
rwt_status rwt_rewrite_symbolic(const rwt_csr* L, const int32_t* d_level,
                                const int32_t* d_set_rows, const int32_t* d_targets,
                                int32_t m, void* d_ws, size_t ws_bytes,
                                int32_t* d_rowptr_out, int32_t* d_cptr_out,
                                int64_t* h_sizes, rwt_stream_t stream);
rwt_status rwt_rewrite_numeric(const rwt_csr* L, const int32_t* d_level,
                               const int32_t* d_set_rows, const int32_t* d_targets,
                               int32_t m, const void* d_B, int32_t k, int64_t ldb,
                               const rwt_csr* Lp, void* d_Bp, int64_t ldbp,
                               int32_t* d_crow, int32_t* d_ccol, void* d_cval,
                               void* d_ws, size_t ws_bytes, rwt_stream_t stream);

/* ------------------------------------------------------------------------
 * Solve plans.  A plan holds the analysis of one matrix, the transposed
 * pattern for the adjoint, and the execution schedule:
 *   RWT_ALGO_LEVEL    level-scheduled: the rows of a level in parallel, a
 *                     device-wide barrier between levels (Section 2.1);
 *                     runs of narrow levels go to one workgroup with the x
 *                     values of the run staged in LDS;
 *   RWT_ALGO_SYNCFREE synchronization-free (Section 7): row blocks claimed
 *                     in row order, each block solved level by level in
 *                     LDS, waiting on per-row readiness in HBM for
 *                     dependencies outside the block; k right-hand sides
 *                     are split into chains of rhs_chunk columns that run
 *                     concurrently (each chain is a full sync-free solve);
 *   RWT_ALGO_WALK     row-order walk (a synchronization-free schedule): one
 *                     wavefront per right-hand-side column solves the rows
 *                     in order, 64 at a time, resolving the dependencies
 *                     inside each chunk of 64 rows in rounds of register
 *                     ballots, one per link of the chunk's longest internal
 *                     dependency chain; suits deep DAGs whose consecutive
 *                     rows seldom depend on each other (the plan reports
 *                     the mean rounds per chunk in rwt_plan_info.chunk_rounds);
 *   RWT_ALGO_AUTO     autotuned: level-scheduled and sync-free are timed on
 *                     the plan's matrix, and the walk too when the chunks
 *                     need at most 12 rounds on average; the fastest is kept.
 * Unless fixed by the options, the sync-free block size, RHS chunk and
 * staging of outside values are chosen by timing solves on the plan's own
 * matrix (min(kmax, 64) columns).
 * The plan keeps pointers to L (pattern and values): the caller keeps them
 * alive and may change the values between solves.  The plan's device
 * state lives in the caller's workspace (rwt_plan_ws bytes).
 * ---------------------------------------------------------------------- */
typedef enum {
    RWT_ALGO_AUTO = 0,
    RWT_ALGO_LEVEL = 1,
    RWT_ALGO_SYNCFREE = 2,
    RWT_ALGO_WALK = 3
} rwt_algo;

typedef struct {
    rwt_algo algo;            /* forward and transposed solves */
    int32_t block_rows;       /* sync-free rows per block (0: choose; else at most 2^20, lowered to fit LDS) */
    int32_t lanes_per_row;    /* 0: choose from the mean row length; else 1..64, power of 2 */
    int32_t narrow_rows;      /* level-scheduled: levels up to this many rows run on one workgroup (-1: choose) */
    int32_t kmax;             /* largest number of right-hand sides solved at once (>=1) */
    int32_t watchdog_ms;      /* bound on any device wait (0: 5000 ms) */
    int32_t rhs_chunk;        /* sync-free columns per chain: 0 choose, else 1..4 */
    int32_t tune_cols;        /* columns the autotuner solves with: 0 min(kmax, 64), else 1..kmax */
    int32_t stage_outside;    /* sync-free, whether the helper waves prefetch the x values a block
                                 reads from earlier blocks: 0 choose by timing both, 1 yes, 2 no
                                 (the solving lanes then load them when they need them) */
} rwt_plan_opts;

typedef struct rwt_plan rwt_plan;

typedef struct {
    rwt_level_stats stats;
    rwt_algo algo_fwd;
    rwt_algo algo_bwd;
    int32_t block_rows;
    int32_t lanes_per_row;
    int32_t narrow_rows;
    int32_t num_blocks;
    int32_t grid;             /* workgroups of the persistent launches */
    int32_t rhs_chunk;        /* sync-free right-hand-side columns per chain */
    int32_t stage_outside;    /* 1 or 2, as in rwt_plan_opts: what the plan uses */
    double tuned_ms_level;    /* autotuner measurements (0 when not tuned); the
                                 level-scheduled figure is its warm-up run alone
                                 when that run took over four times the best of
                                 the other two */
    double tuned_ms_syncfree;
    double tuned_ms_walk;
    double chunk_rounds;      /* mean over 64-row chunks of the rounds the walk needs */
} rwt_plan_info;

rwt_status rwt_plan_ws(const rwt_csr* L, const rwt_plan_opts* opts, size_t* h_bytes);
rwt_status rwt_plan_create(const rwt_csr* L, const rwt_plan_opts* opts, void* d_ws,
                           size_t ws_bytes, rwt_plan** out, rwt_stream_t stream);
rwt_status rwt_plan_get_info(const rwt_plan* plan, rwt_plan_info* h_info);
/* device arrays owned by the plan's workspace: level[n], perm[n], level_ptr[D+1] */
rwt_status rwt_plan_levels(const rwt_plan* plan, const int32_t** d_level,
                           const int32_t** d_perm, const int32_t** d_level_ptr);
rwt_status rwt_plan_destroy(rwt_plan* plan);

/* ------------------------------------------------------------------------
 * Tall-block row order (host code, no device work; not in the paper: a
 * schedule aid for the sync-free solve of Section 7).  The sync-free solve
 * walks blocks of consecutive rows, and a dependency chain that leaves its
 * block at every level pays a cross-workgroup hand-off per level.  This
 * returns a topological order of L's rows in which consecutive rows form
 * tiles of whole chains: chains follow each row's dependency one level
 * below (Section 2.1 levels), chains of chains do the same on the chain
 * heads, and a tile is a positions along a chain of chains by b chains of
 * chains.
 *   h_rowptr[n+1], h_colidx[nnz]: L's pattern in host memory (entries of a
 *     row below the diagonal, the diagonal last; values are not read);
 *   a, b: tile shape (0: 4 and 8);
 *   h_perm[n] (caller's host buffer, out): new -> old row numbers.  The
 *     matrix P L P^T, entry (i, j) = L[perm[i]][perm[j]], is lower
 *     triangular: solve it with b'[i] = b[perm[i]] and set x[perm[i]] = x'[i].
 * For a rewritten factor L' = M L compute the order on L: rewriting only
 * adds dependencies from the transitive closure of L's DAG, so L's order
 * stays topological for L' and keeps its tiles (the rewritten rows change
 * the chains when the order is computed on L' itself).
 * Errors: RWT_ERR_INVALID_ARG (null pointer, negative n, a or b, rowptr[0]
 * not 0), RWT_ERR_MISSING_DIAG (a row empty or not ending at its
 * diagonal), RWT_ERR_NOT_LOWER (a column outside [0, row)); h_perm is then
 * unspecified.
 * ---------------------------------------------------------------------- */
rwt_status rwt_tall_block_order(int32_t n, const int32_t* h_rowptr, const int32_t* h_colidx,
                                int32_t a, int32_t b, int32_t* h_perm);

/* Forward solve L X = B (Section 2.1).  k <= kmax.  d_X may equal d_B
 * (in place).  A watchdog expiry returns RWT_ERR_DEADLOCK (synchronizing
 * only when it must report). */
rwt_status rwt_solve(const rwt_plan* plan, const void* d_B, int32_t k, int64_t ldb,
                     void* d_X, int64_t ldx, rwt_stream_t stream);

/* Transposed solve L^T Y = G (the adjoint: upper triangular, levels taken
 * in reverse order).  d_Y may equal d_G. */
rwt_status rwt_solve_transpose(const rwt_plan* plan, const void* d_G, int32_t k, int64_t ldg,
                               void* d_Y, int64_t ldy, rwt_stream_t stream);

/* Test aid for the watchdog path of the sync-free solves (Section 7: a
 * reader spins until its dependency is published).  Runs rwt_solve but
 * never publishes row `row`'s values to d_X (the row is still solved and
 * its block reads it from LDS), so every reader outside that block waits
 * until the plan's watchdog (rwt_plan_opts.watchdog_ms) expires; every wait
 * then ends, the kernel exits, rwt_plan_check reports RWT_ERR_DEADLOCK and
 * d_X holds unspecified values.  The next rwt_solve on the plan is
 * unaffected.  Errors: RWT_ERR_INVALID_ARG for a row outside [0, n), and
 * those of rwt_solve. */
rwt_status rwt_solve_withhold(const rwt_plan* plan, int32_t row, const void* d_B, int32_t k,
                              int64_t ldb, void* d_X, int64_t ldx, rwt_stream_t stream);

/* Device error word of the last solve on this plan (RWT_OK or
 * RWT_ERR_DEADLOCK).  Synchronizes the stream. */
rwt_status rwt_plan_check(const rwt_plan* plan, rwt_stream_t stream);

/* ------------------------------------------------------------------------
 * Upper-triangular solves and the L-then-U pair: applying an incomplete LU
 * preconditioner M = L U in an iterative solver means one forward solve
 * with L and one backward solve with U per iteration, which is the use the
 * cost of rewriting is amortized over (a few hundred iterations).
 *
 * U: CSR, each row holding its diagonal first, then strictly ascending
 * columns above it (FP64 or FP32 values, non-zero diagonal).  The upper
 * plan solves through the lower matrix J U J (J reverses the index order),
 * with every schedule and the autotuner of rwt_plan_create (opts as there).
 * rwt_upper_create checks U (synchronizes): a violation is reported with
 * the status of the matching lower check -- RWT_ERR_NOT_LOWER for an entry
 * below the diagonal or a column out of range, RWT_ERR_UNSORTED_OR_DUP,
 * RWT_ERR_MISSING_DIAG (first entry not the diagonal), RWT_ERR_ZERO_DIAG --
 * and the U row in rwt_last_error_string; RWT_ERR_INVALID_ARG for row
 * pointers that are not a CSR index.  The plan keeps U's pointers and a
 * copy of its values in the reversed order: after changing U's values call
 * rwt_upper_refresh.  Workspace: rwt_upper_ws bytes (holds the reversed
 * pattern, an n x kmax block and the inner plan).
 *
 * rwt_upper_solve:           X = U^{-1} B   (backward substitution)
 * rwt_upper_solve_transpose: Y = U^{-T} G
 * rwt_solve_pair:            X = U^{-1} (L^{-1} B), L a lower plan of the
 *                            same size and value type; k <= both kmax.
 * d_X may equal d_B.  Dense blocks column-major, ld >= n.
 * ---------------------------------------------------------------------- */
typedef struct rwt_upper rwt_upper;

rwt_status rwt_upper_ws(const rwt_csr* U, const rwt_plan_opts* opts, size_t* h_bytes);
rwt_status rwt_upper_create(const rwt_csr* U, const rwt_plan_opts* opts, void* d_ws,
                            size_t ws_bytes, rwt_upper** out, rwt_stream_t stream);
rwt_status rwt_upper_refresh(rwt_upper* up, rwt_stream_t stream);
rwt_status rwt_upper_get_info(const rwt_upper* up, rwt_plan_info* h_info);
/* Levels of the backward substitution: the device arrays of the plan of
 * J U J (as rwt_plan_levels), in the reversed numbering -- entry i' is U's
 * row n-1-i'. */
rwt_status rwt_upper_levels(const rwt_upper* up, const int32_t** d_level, const int32_t** d_perm,
                            const int32_t** d_level_ptr);
rwt_status rwt_upper_solve(const rwt_upper* up, const void* d_B, int32_t k, int64_t ldb,
                           void* d_X, int64_t ldx, rwt_stream_t stream);
rwt_status rwt_upper_solve_transpose(const rwt_upper* up, const void* d_G, int32_t k,
                                     int64_t ldg, void* d_Y, int64_t ldy, rwt_stream_t stream);
rwt_status rwt_solve_pair(const rwt_plan* L, const rwt_upper* U, const void* d_B, int32_t k,
                          int64_t ldb, void* d_X, int64_t ldx, rwt_stream_t stream);
/* device error word of the last solve (as rwt_plan_check; synchronizes) */
rwt_status rwt_upper_check(const rwt_upper* up, rwt_stream_t stream);
rwt_status rwt_upper_destroy(rwt_upper* up);

/* ------------------------------------------------------------------------
 * Adjoint helpers.  With X = L^{-1} B, G = dLoss/dX and the rewritten system
 * L' = M L, B' = M B (M = I - C):  Y = L'^{-T} G, grad_B = M^T Y = Y - C^T Y
 * and grad_L = -grad_B X^T restricted to L's pattern.
 *
 * rwt_apply_MT: d_out = d_Y - C^T d_Y for the multipliers of a rewrite
 * (nC entries d_crow/d_ccol/d_cval, grouped by d_crow ascending as written
 * by rwt_rewrite_numeric).  Deterministic (no atomics): the workspace
 * (rwt_apply_MT_ws bytes) holds C^T, built by the call.  d_out may not alias
 * d_Y.
 * rwt_grad_vals: d_gvals[p] = -sum_q d_gB[row_p, q] * d_X[col_p, q] for every
 * stored entry p of the pattern of L (diagonal included).
 * ---------------------------------------------------------------------- */
/* rwt_apply_M: d_out = M d_B = d_B - C d_B for the multipliers of a rewrite
 * (grouped by d_crow ascending, as rwt_rewrite_numeric writes them; each
 * row's substitutions applied in their order, so the result equals the B'
 * of the rewrite bit for bit).  This is the right-hand side transform of
 * the rewritten system for a new B: solving L' X = M B gives L^{-1} B, e.g.
 * in each application of a preconditioner with the rewritten factor.
 * Workspace: rwt_apply_M_ws(n) bytes (row offsets of the multipliers,
 * rebuilt by every call).  d_out may not alias d_B. */
rwt_status rwt_apply_M_ws(int32_t n, size_t* h_bytes);
rwt_status rwt_apply_M(int32_t n, int64_t nC, const int32_t* d_crow, const int32_t* d_ccol,
                       const void* d_cval, rwt_dtype dt, const void* d_B, int32_t k,
                       int64_t ldb, void* d_out, int64_t ldo, void* d_ws, size_t ws_bytes,
                       rwt_stream_t stream);
/* rwt_apply_M_noalloc: rwt_apply_M for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, result and
 * errors as rwt_apply_M, without d_ws: the multipliers' row offsets go to a
 * library-owned device array of RWT_APPLY_M_NOALLOC_MAX_N + 1 int32 entries
 * (16 MiB, one copy per GPU the library runs on, held until the process
 * ends; its device address is looked up on the first call on each device,
 * which must be the current device).  n above RWT_APPLY_M_NOALLOC_MAX_N
 * returns RWT_ERR_TOO_LARGE before any launch.  Every call on one GPU uses
 * that GPU's one array: calls that overlap on one GPU (other streams, other
 * host threads) race and must be serialized by the caller.  Nothing is
 * allocated or freed by the call. */
#define RWT_APPLY_M_NOALLOC_MAX_N (1 << 22)
rwt_status rwt_apply_M_noalloc(int32_t n, int64_t nC, const int32_t* d_crow,
                               const int32_t* d_ccol, const void* d_cval, rwt_dtype dt,
                               const void* d_B, int32_t k, int64_t ldb, void* d_out, int64_t ldo,
                               rwt_stream_t stream);
rwt_status rwt_apply_MT_ws(int32_t n, int64_t nC, size_t* h_bytes);
rwt_status rwt_apply_MT(int32_t n, int64_t nC, const int32_t* d_crow, const int32_t* d_ccol,
                        const void* d_cval, rwt_dtype dt, const void* d_Y, int32_t k, int64_t ldy,
                        void* d_out, int64_t ldo, void* d_ws, size_t ws_bytes,
                        rwt_stream_t stream);
/* The two halves of rwt_apply_MT, for repeated use with one multiplier
 * pattern (the pattern of C is structural: it does not change when the
 * rewrite's numeric part is re-run).  rwt_apply_MT_prepare builds the C^T
 * ordering from d_ccol into the workspace; rwt_apply_MT_apply then applies
 * Y - C^T Y with any values d_cval, reading that ordering.  Same sizes,
 * errors and workspace (rwt_apply_MT_ws bytes) as rwt_apply_MT; the caller
 * keeps the workspace untouched between the two. */
rwt_status rwt_apply_MT_prepare(int32_t n, int64_t nC, const int32_t* d_ccol, void* d_ws,
                                size_t ws_bytes, rwt_stream_t stream);
rwt_status rwt_apply_MT_apply(int32_t n, int64_t nC, const int32_t* d_crow, const void* d_cval,
                              rwt_dtype dt, const void* d_Y, int32_t k, int64_t ldy, void* d_out,
                              int64_t ldo, const void* d_ws, size_t ws_bytes,
                              rwt_stream_t stream);
rwt_status rwt_grad_vals(const rwt_csr* L, const void* d_gB, int64_t ldg, const void* d_X,
                         int64_t ldx, int32_t k, void* d_gvals, rwt_stream_t stream);

/* ------------------------------------------------------------------------
 * Rewrite-list generator: the environment of Section 4.1 run with a fixed
 * policy in place of the learned one, one environment per parameter set,
 * all over one matrix in one launch.  Each returns a rewriting list of
 * <node, source level, target level> triplets (Algorithm 1) that
 * rwt_rewrite_* or a batch's candidate lists take directly.
 *
 * State (Section 4.1, updated per move without touching the DAG): the level
 * of every row and, per level, its cost (sum of 2*nnz_i - 1; a moved row
 * keeps its original cost), row count and indegree (sum of nnz_i - 1).
 * Level numbers never change; an emptied level is skipped by the searches.
 * thr = ALC * (1 + alpha * max(0, 1 - CV)) from the input's ALC and CV,
 * fixed for the run; thin = non-empty and cost < thr.
 * One step:
 *   source  the thin level >= 1 that never received a row and was never
 *           rejected, with the fewest rows (ties: lower level);
 *   node    its row with the fewest dependencies (ties: lower row),
 *           Section 4.3;
 *   target  Algorithm 1 with equal affinities: p = nearest non-empty level
 *           above the source; p == 0: level 0 if thin, else reject; p > 0:
 *           the nearest thin level at or above p, else p itself; reject when
 *           source - target > max_dist (MAX_REWRITE_DISTANCE).  A rejected
 *           source is not chosen again;
 *   move    the row joins the target level; both levels' sums change; the
 *           triplet is appended.
 * Before each step, in this order: stop RWT_GEN_THIN when the initial thin
 * count T0 > 0 and thin/T0 < thin_stop; RWT_GEN_MOVES at the move limit;
 * RWT_GEN_STEPS at the step limit (rejected steps count); RWT_GEN_NO_SOURCE
 * when no source is left.
 *
 * Inputs: L (pattern only), and from rwt_analyze of L: d_level[n],
 * d_level_ptr[D+1], d_cost[D], d_stats (device) and D = num_levels.
 * h_params[num_env] (host).  Outputs (device, caller-allocated): for
 * environment e, moves q < d_res[e].moves at d_mv_row/src/tgt[e*cap + q] in
 * move order; d_res[num_env]; optionally (nullable) the final per-level
 * sums d_lev_cost/d_lev_rows/d_lev_deps[e*D + l].  Workspace:
 * rwt_generate_ws bytes.  Asynchronous on the stream (the parameters are
 * copied from the host before return).
 * ---------------------------------------------------------------------- */
typedef struct {
    double alpha;        /* threshold relaxation, >= 0 (the paper uses 1.0) */
    double thin_stop;    /* stop below this thin-level ratio (the paper: 0.02) */
    int32_t max_dist;    /* largest source - target distance, >= 0 */
    int32_t max_moves;   /* 0: cap */
    int32_t max_steps;   /* 0: max(2 D, 3 * 2048) */
    int32_t pad_;
} rwt_gen_params;

typedef enum {
    RWT_GEN_NO_SOURCE = 0,
    RWT_GEN_THIN = 1,
    RWT_GEN_MOVES = 2,
    RWT_GEN_STEPS = 3
} rwt_gen_stop;

typedef struct {
    int32_t moves;
    int32_t steps;       /* moves + rejected */
    int32_t stop;        /* rwt_gen_stop */
    int32_t levels;      /* non-empty levels at the end */
    int32_t thin;        /* thin levels at the end */
    int32_t thin0;       /* thin levels at the start */
    int32_t rejected;
    int32_t pad_;
    double threshold;
    uint64_t S1;         /* sum of the non-empty levels' costs */
    uint64_t S2_lo;      /* sum of their squares, 128 bit */
    uint64_t S2_hi;
    double cv;           /* their CV, as in rwt_level_stats */
} rwt_gen_result;

rwt_status rwt_generate_ws(int32_t n, int32_t num_levels, int32_t num_env, size_t* h_bytes);
rwt_status rwt_generate(const rwt_csr* L, const int32_t* d_level, const int32_t* d_level_ptr,
                        const int64_t* d_cost, const rwt_level_stats* d_stats,
                        int32_t num_levels, int32_t num_env, const rwt_gen_params* h_params,
                        int32_t cap, int32_t* d_mv_row, int32_t* d_mv_src, int32_t* d_mv_tgt,
                        rwt_gen_result* d_res, int64_t* d_lev_cost, int32_t* d_lev_rows,
                        int64_t* d_lev_deps, void* d_ws, size_t ws_bytes,
                        rwt_stream_t stream);

/* Candidate row sets from generated lists, in the form the rewrite and the
 * batch take: d_cand_ptr[num_env+1] (exclusive offsets of each
 * environment's moves), d_cand_rows / d_cand_targets[num_env*cap] (each
 * environment's moved rows ascending, with their target levels; targets
 * nullable).  No host synchronization (graph-capturable).  Workspace:
 * rwt_gen_rowsets_ws bytes; num_env*cap < 2^31. */
rwt_status rwt_gen_rowsets_ws(int32_t num_env, int32_t cap, size_t* h_bytes);
rwt_status rwt_gen_rowsets(int32_t n, int32_t num_env, int32_t cap, const rwt_gen_result* d_res,
                           const int32_t* d_mv_row, const int32_t* d_mv_tgt,
                           int32_t* d_cand_ptr, int32_t* d_cand_rows, int32_t* d_cand_targets,
                           void* d_ws, size_t ws_bytes, rwt_stream_t stream);

/* ------------------------------------------------------------------------
 * Environment step (Sections 4.1-4.5, Algorithms 1 and 2) for many
 * environments over one matrix, driven by the caller's policy: every call
 * of rwt_env_step applies one action (a source level) per environment and
 * returns its reward; rwt_env_observe writes the observation of Table 1
 * and the action mask of Section 4.3.  The rewriting list of each
 * environment grows in the caller's move arrays.
 *
 * State (Section 4.1; the DAG is never modified): the level of every row
 * and, per level, its cost (sum of 2*nnz_i - 1; a moved row keeps its
 * original cost), row count and dependency sum; per level also whether it
 * ever received a row, its initial size and first-touch step (abandonment)
 * and the steps of its last choice as source and of its last received row
 * (affinities, Section 4.2).  thr = ALC * (1 + alpha * max(0, 1 - CV)) of
 * the input, fixed; thin = non-empty and cost < thr; levels and CV count
 * the non-empty levels.
 *
 * One step with action a (readings of what the paper leaves open):
 *   validity  1 <= a < D and level a non-empty (the mask heuristics shape
 *             the policy's mask only).  An invalid action, or one that
 *             Algorithm 1 rejects, changes only the step count; reward
 *             -reward_alpha;
 *   node      the row of level a with the fewest dependencies (ties: lower
 *             row), rows that moved in included (Section 4.3);
 *   target    Algorithm 1: p = nearest non-empty level above a; p == 0:
 *             level 0 if thin, else reject; p > 0: among the search_window
 *             nearest thin levels at or above p, the one that most recently
 *             received a row (never: lowest; ties: the nearest); with none,
 *             p when the source is thin, else reject; reject when a - t >
 *             max_dist;
 *   reward    Algorithm 2 with dCV = CV before - CV after:
 *             r_cv = -reward_alpha if dCV < -eps, D0*dCV if dCV > eps, else 0;
 *             s = ln(size + 2) with the source's rows before the move;
 *             r_cp = reward_alpha (D0/levels after)(1 + 1/s) when the source
 *             emptied, reward_alpha/s when it was thin, else
 *             -reward_alpha (1 + s);
 *             r_rwdist = log1p(thd - d)/D0 if d < thd else -log1p(d - thd)/D0,
 *             d = a - t, thd = dist_threshold;
 *             r_abandon for the previous move's source A != a: if A ever
 *             received a row, its initial size becomes its current size and
 *             its first touch 0, no penalty; none if A is empty, or if a
 *             level >= 1 with one row exists and A is thin; else
 *             -(rows_A/(init_A + 1)) * log1p(step - first touch of A);
 *             reward = 0.80 r_cv + 0.80 r_cp + 0.05 r_rwdist + 0.50 r_abandon
 *             (the weights of Section 4.4); D0 = initial level count.
 *   end       checked after reset and after every step, in this order:
 *             RWT_GEN_THIN when T0 > 0 and thin/T0 < thin_stop;
 *             RWT_GEN_MOVES after cap moves; RWT_GEN_STEPS after max_steps
 *             steps (0 = max(2 D, 6144)); RWT_GEN_NO_SOURCE when only level
 *             0 is non-empty.  Later actions are ignored (reward 0).
 *
 * Workspace: rwt_env_ws bytes, owned by the caller and kept between calls;
 * rwt_env_init builds the tables from the analysis of L (d_level[n],
 * d_level_ptr[D+1], d_cost[D], d_stats, D = num_levels; device) and resets
 * every environment; it synchronizes the stream before returning.  Every
 * later call must pass the same n, num_levels, num_env, cap and workspace:
 * the kernels check them against the workspace and do nothing (step:
 * outcome RWT_ENV_ERROR) on a mismatch.  Calls on one workspace must not
 * overlap.  Sizes: n >= 1, 1 <= num_levels <= n, num_env >= 1, cap >= 1.
 * ---------------------------------------------------------------------- */
typedef struct {
    double alpha;            /* threshold relaxation, >= 0 (the paper: 1.0) */
    double thin_stop;        /* episode end below this thin ratio (0.02) */
    double reward_alpha;     /* alpha of Algorithm 2, >= 0 */
    double eps;              /* dead band of dCV, >= 0 */
    double decay;            /* affinity decay per step, in (0, 1) */
    int32_t max_dist;        /* MAX_REWRITE_DISTANCE, >= 0 */
    int32_t search_window;   /* SEARCH_WINDOW (the paper: 5), >= 1 */
    int32_t dist_threshold;  /* threshold of r_rwdist, >= 0 */
    int32_t max_steps;       /* truncation; 0 = max(2 D, 6144) */
    int32_t stall_steps;     /* mask to keep_top after this many steps
                                without a collapse; 0 = off */
    int32_t keep_top;        /* X of Section 4.3, >= 1 */
} rwt_env_params;

typedef enum {
    RWT_ENV_MOVED = 0,
    RWT_ENV_INVALID = 1,
    RWT_ENV_REJECTED = 2,   /* Algorithm 1 found no target */
    RWT_ENV_IGNORED = 3,    /* the episode had ended */
    RWT_ENV_ERROR = 4       /* workspace mismatch or corrupt state */
} rwt_env_outcome;

typedef struct {
    int32_t outcome;     /* rwt_env_outcome */
    int32_t node;        /* the row chosen (moved or rejected), else -1 */
    int32_t src;         /* the action when it was valid, else -1 */
    int32_t tgt;         /* target level of a move, else -1 */
    int32_t collapsed;   /* the source emptied */
    int32_t done;        /* -1 running, else an rwt_gen_stop */
    int32_t steps, moves, levels, thin, thin0, pad_;
    double reward;
    double r_cv, r_cp, r_rwdist, r_abandon;   /* 0 unless moved */
    double cv;           /* CV of the non-empty levels' costs after the step */
    double cv_rows;      /* CV of their row counts */
} rwt_env_result;

rwt_status rwt_env_ws(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                      size_t* h_bytes);
rwt_status rwt_env_init(const rwt_csr* L, const int32_t* d_level, const int32_t* d_level_ptr,
                        const int64_t* d_cost, const rwt_level_stats* d_stats,
                        int32_t num_levels, int32_t num_env, int32_t cap,
                        const rwt_env_params* h_params, void* d_ws, size_t ws_bytes,
                        rwt_stream_t stream);
/* Reset the environments e with d_which[e] != 0 (device, nullable: all). */
rwt_status rwt_env_reset(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                         const uint8_t* d_which, void* d_ws, size_t ws_bytes,
                         rwt_stream_t stream);
/* d_action[num_env] (device); d_res[num_env]; move q of environment e is
 * written to d_mv_row/src/tgt[e*cap + q] (the same arrays at every step
 * since the environment's reset).  Asynchronous. */
rwt_status rwt_env_step(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                        const int32_t* d_action, rwt_env_result* d_res, int32_t* d_mv_row,
                        int32_t* d_mv_src, int32_t* d_mv_tgt, void* d_ws, size_t ws_bytes,
                        rwt_stream_t stream);
/* Observation (each output nullable, device, float32 / uint8):
 *   d_obs_level[(e*6 + f)*D + l], f = 0..5: cost/ALC, rows/ARL, source
 *     affinity, target affinity, completion ratio 1 - rows/(init + 1),
 *     thin (1/0); affinity = decay^(steps - stamp), 0 if never, -1 when the
 *     level is empty or (source) ever received a row or (target) not thin;
 *   d_obs_global[e*9 + g]: CV of level costs, 1 (its reference), CV of rows
 *     per level, 1, levels/n, moves/n (rewrite ratio), thin/T0 (0 if T0 =
 *     0), levels/D0 (critical-path ratio), thin/levels;
 *   d_mask[e*D + l]: 1 for levels >= 1 that are non-empty while the episode
 *     runs; only the previous source when it has one row left; otherwise,
 *     after stall_steps steps without a collapse, only the keep_top of
 *     highest source affinity (levels that received rows rank lowest, ties
 *     to the lower level).  Asynchronous. */
rwt_status rwt_env_observe(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                           float* d_obs_level, float* d_obs_global, uint8_t* d_mask,
                           const void* d_ws, size_t ws_bytes, rwt_stream_t stream);
/* rwt_env_step followed by rwt_env_observe, in one launch: the same
 * results, moves, observation and mask as the two calls (observation
 * outputs nullable). */
rwt_status rwt_env_step_observe(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                                const int32_t* d_action, rwt_env_result* d_res,
                                int32_t* d_mv_row, int32_t* d_mv_src, int32_t* d_mv_tgt,
                                float* d_obs_level, float* d_obs_global, uint8_t* d_mask,
                                void* d_ws, size_t ws_bytes, rwt_stream_t stream);
/* Per-level state d_cost/d_rows/d_deps[e*D + l] (device, each nullable). */
rwt_status rwt_env_levels(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                          int64_t* d_cost, int32_t* d_rows, int64_t* d_deps, const void* d_ws,
                          size_t ws_bytes, rwt_stream_t stream);

/* ------------------------------------------------------------------------
 * Batched launch: many matrices of uneven size, each with its own block of
 * right-hand sides, plus many candidate rewrite sets (rewriting lists in
 * the sense of Algorithm 1, one per environment step of the paper's agent)
 * whose level statistics are computed -- all in one persistent kernel,
 * preceded by a few setup kernels, launched together (optionally replayed
 * from a captured hipGraph).
 *
 * Per matrix m: L (FP64 values), B / X (k columns; k may be 0 for
 * analysis-only matrices).  Its solve runs in sync-free row blocks of the
 * largest size whose x values fit in LDS (the whole matrix in one
 * workgroup, level after level, when it fits), one column per chain,
 * unless block_rows fixes the block size.
 * Candidate levels are computed either as a chain of row-block tasks (the
 * blocks of the matrix's solve schedule, waiting on each other's levels)
 * or by one workgroup sweeping the original levels in order (every row of
 * an original level at once: a rewritten row's new dependencies lie on
 * earlier original levels too).  With cand_mode 0 a matrix's candidates
 * take the sweep when its block chain has at least four times as many
 * level steps as the matrix has levels (wide levels), else the chain
 * (always the chain for a matrix of 2^23 levels or more).  Sweeps of
 * consecutive candidates of one matrix run up to eight to a workgroup,
 * their levels interleaved row by row, so that one read of a dependency's
 * levels serves all of them.
 * Per candidate c: the matrix h_cand_mat[c] and the rows
 * d_cand_rows[d_cand_ptr[c] .. d_cand_ptr[c+1]) (strictly ascending) with
 * targets d_cand_targets (NULL: level - 1).  Each launch recomputes, for
 * every candidate, the levels of the rewritten matrix L' and its statistics
 * (level count, S1, exact S2, CV of level costs) -- L' itself is not formed.
 * The row lists (and d_cand_ptr) may change between launches within
 * cand_rows_cap rows and pattern_cap rewritten-row entries.
 *
 * The batch keeps pointers to every caller array; the workspace
 * (rwt_batch_ws bytes) holds the per-matrix plans and all scratch.
 * Invalid candidate row lists are skipped (statistics flagged invalid) and
 * reported by rwt_batch_stats as RWT_ERR_BAD_ROWSET.
 * ---------------------------------------------------------------------- */
typedef struct {
    rwt_csr L;            /* device, FP64 values */
    const void* B;        /* device, k columns (ldb) */
    void* X;              /* device, k columns (ldx) */
    int32_t k;
    int32_t block_rows;   /* solve row-block size; 0: the largest that fits the LDS
                             budget (fewer level steps for the solve and the
                             candidate chains that share its blocks) */
    int64_t ldb;
    int64_t ldx;
} rwt_batch_matrix;

typedef struct {
    int32_t count;                      /* matrices */
    int32_t num_cand;                   /* candidate rewrite sets */
    const rwt_batch_matrix* mats;       /* host array of count */
    const int32_t* h_cand_mat;          /* host, num_cand */
    const int32_t* d_cand_ptr;          /* device, num_cand + 1 */
    const int32_t* d_cand_rows;         /* device */
    const int32_t* d_cand_targets;      /* device or NULL */
    int32_t cand_rows_cap;              /* capacity of the concatenated row lists */
    int32_t pattern_cap;                /* capacity of rewritten-row patterns (0: 64 per row).
                                           With at least 48 per row of cand_rows_cap they are
                                           built in one pass: a fixed slot of 32 entries per
                                           row, longer rows in the rest of the capacity;
                                           otherwise in two (lengths, then patterns) */
    int32_t watchdog_ms;
    int32_t cand_mode;                  /* candidate levels: 0 choose per matrix, 1 row-block
                                           chains, 2 one level sweep per candidate, 3 the
                                           row-order walk (one wave per candidate) */
} rwt_batch_desc;

typedef struct {
    int32_t num_levels;
    int32_t valid;        /* 0: the candidate's row list was rejected */
    uint64_t S1;
    uint64_t S2_lo;
    uint64_t S2_hi;
    double cv;
} rwt_cand_stats;

typedef struct {
    int32_t tasks;        /* tasks of the persistent launch */
    int32_t solve_tasks;
    int32_t grid;
    int32_t captured;     /* a graph is instantiated */
    double create_ms;
    int32_t sweep_cands;  /* candidates scored by one level sweep */
    int32_t pattern_slot; /* entries of a row's fixed pattern slot (one-pass patterns),
                             0 when the patterns take two passes */
} rwt_batch_info;

typedef struct rwt_batch rwt_batch;

rwt_status rwt_batch_ws(const rwt_batch_desc* desc, size_t* h_bytes);
rwt_status rwt_batch_create(const rwt_batch_desc* desc, void* d_ws, size_t ws_bytes,
                            rwt_batch** out, rwt_stream_t stream);
rwt_status rwt_batch_run(rwt_batch* batch, rwt_stream_t stream);
/* rwt_batch_run in its two parts, enqueued one after the other on one
 * stream: the setup kernels (launch epoch, resets, candidate checks and
 * the batched symbolic rewrite) and then the persistent kernel alone (so
 * that a caller can time it with events recorded in between).  Calling
 * rwt_batch_run_main without the setup of the same launch before it is an
 * error the library cannot detect. */
rwt_status rwt_batch_run_setup(rwt_batch* batch, rwt_stream_t stream);
rwt_status rwt_batch_run_main(rwt_batch* batch, rwt_stream_t stream);
/* stream must not be the legacy default stream (capture needs a real stream) */
rwt_status rwt_batch_capture(rwt_batch* batch, rwt_stream_t stream);
rwt_status rwt_batch_launch(rwt_batch* batch, rwt_stream_t stream);
rwt_status rwt_batch_stats(const rwt_batch* batch, rwt_cand_stats* h_out, rwt_stream_t stream);
rwt_status rwt_batch_get_info(const rwt_batch* batch, rwt_batch_info* h_info);
rwt_status rwt_batch_plan(const rwt_batch* batch, int32_t m, const rwt_plan** out);
rwt_status rwt_batch_destroy(rwt_batch* batch);

/* ------------------------------------------------------------------------
 * Measurement of the hand-off that bounds sync-free schedules from below:
 * one workgroup publishes a value with a relaxed device-scope store, a
 * second finds it with relaxed device-scope loads (the readiness mechanism
 * of the solves).  Two workgroups exchange `rounds` values back and forth;
 * *h_ns_one_way = elapsed / (2 rounds).  A latency floor of a solve with D
 * dependent levels crossing workgroups is about D times this.  Every wait
 * is bounded (100 ms in all: RWT_ERR_DEADLOCK).  Workspace:
 * rwt_probe_handoff_ws(rounds) bytes.  Synchronizes.
 * ---------------------------------------------------------------------- */
size_t rwt_probe_handoff_ws(int32_t rounds);
rwt_status rwt_probe_handoff(int32_t rounds, void* d_ws, size_t ws_bytes, double* h_ns_one_way,
                             rwt_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* RWTRSV_H */
