/*
 * lpgpu: dense full-tableau primal simplex on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Mamalis & Perlitis, Section III):
 *     maximise c^T x  subject to  A x <= b,  x >= 0,  with b >= 0,
 * solved by the standard full-tableau method: the tableau of Table I with the
 * slack basis (Initialization Step); Step 1 picks the entering column with the
 * most negative objective-row entry; Step 2 the leaving row by the minimum
 * ratio test; Step 3 pivots the whole tableau; the loop stops at optimality or
 * unboundedness (Iterate/Finalization Step).
 *
 * Arithmetic contract (binary64 throughout, identical in every mode):
 *   - tableau T has m+1 rows and W = n+m+1 columns; the z column of Table I
 *     is left out (it stays the unit vector e_0); column W-1 is the RHS;
 *   - Step 1: q = lowest j in [0, n+m) with the smallest T[0][j]; optimal when
 *     T[0][q] >= -eps_dual;
 *   - Step 2: over rows i in [1, m] with T[i][q] > eps_pivot, the smallest
 *     T[i][W-1] / T[i][q] (IEEE division), lowest i on ties; none: unbounded;
 *   - iteration cap: checked after Step 2; max_pivots pivots done and another
 *     one needed gives LP_ITER_LIMIT;
 *   - Step 3: p = T[r][q]; F = column q before the update; R_j = T[r][j] / p;
 *     T[i][j] = fma(-F_i, R_j, T[i][j]) for i != r; T[r][j] = R_j;
 *   - non-finite values (LP_NUMERICAL): Step 1 stops when row 0 holds a NaN
 *     or its smallest entry is -inf; Step 2 stops when, in some row 1..m,
 *     the entering column holds a value that is not finite or the RHS holds
 *     a NaN (an overflowing ratio is an ordinary infinite ratio).
 * Results: x_j is the RHS of the row where j is basic (0 when nonbasic),
 * y_i = T[0][n+i-1] (the duals), objective = T[0][W-1]. The same LP gives the
 * same pivot sequence alone, in a batch and in the server.
 *
 * Conventions: every function returns an int32 code (LP_OK = 0, negative =
 * error) unless stated. Host arrays are caller-owned and only read during the
 * call (inputs are copied). Pivot logs hold the tableau row r in [1, m] and
 * the column q in [0, n+m). Contexts are not thread-safe; distinct contexts
 * may be used from distinct threads. The server is thread-safe.
 */
#ifndef LPGPU_H
#define LPGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Outcome of a solve (lp_result.status). */
enum {
    LP_OPTIMAL = 0,    /* Step 1 found no entering column */
    LP_UNBOUNDED = 1,  /* Step 2 found no eligible row */
    LP_ITER_LIMIT = 2, /* max_pivots pivots done, another one needed */
    LP_NUMERICAL = 3,  /* Step 1 or Step 2 met a non-finite value (see the contract above) */
    LP_RUNNING = 4,    /* not finished (lp_step budget ran out, or not solved yet) */
    LP_STALLED = 5,    /* a grid-barrier wait of the one-launch decision kernel timed out
                          after all its workgroups had checked in (only with a decide_spin far
                          below the default); the solve was abandoned. A launch whose
                          workgroups cannot all be resident at once (other work holding the
                          compute units) closes its check-in gate instead, writes nothing,
                          and the solve goes on with the barrier-free decision kernels (two
                          launches per pivot, groups of at most 16 pivots): no status, the
                          same pivots and bits; lp_get_info then reports decide_workgroups 0 */
    LP_INFEASIBLE = 6  /* general form: Phase I ended with artificial variables above zero */
};

/* Row senses of the general form (lp_create_general). */
enum { LP_LE = 0, LP_GE = 1, LP_EQ = 2 };

/* Return codes. */
enum {
    LP_OK = 0,
    LP_E_INVAL = -1,   /* NULL pointer, m or n < 1, non-finite input, bad option */
    LP_E_NEG_RHS = -2, /* some b_i < 0: the slack basis is infeasible (the standard-form
                          entry points have no Phase I; lp_create_general has) */
    LP_E_NOMEM = -3,   /* device or host allocation failed */
    LP_E_DEVICE = -4,  /* a HIP call failed; lp_last_error() has the text */
    LP_E_STATE = -5,   /* call out of order (e.g. solution before solve) */
    LP_E_PENDING = -6, /* server result not ready yet */
    LP_E_BUDGET = -7   /* LP larger than the server's memory budget */
};

typedef struct lp_ctx lp_ctx;
typedef struct lp_batch lp_batch;
typedef struct lp_server lp_server;
typedef struct lp_hybrid lp_hybrid;

/*
 * Execution and kernel-shape choices. None of them changes a result: every
 * choice gives the same pivots and bit-identical tableaux. All zero (as
 * lp_tuning_default sets it) means automatic choices throughout.
 */
typedef struct {
    int32_t chunk_pivots;   /* pivots per replay of the captured graph; 0 = auto (4, or one group
                               of fuse_pivots pivots when K > 1) */
    int32_t cols_per_block; /* update kernel: listed columns per workgroup (1, 2, 4, 8, 16; 0 = auto) */
    int32_t plain_launches; /* 1 = launch the kernels directly instead of replaying a captured
                               hipGraph (default 0) */
    int32_t time_kernels;   /* 1 = time every update kernel with HIP events (lp_get_timing); the
                               kernels are then launched directly, not from a graph (default 0) */
    int32_t rows_per_thread;/* update kernel: row pairs per thread and column (1, 2, 4, 8; 0 = auto) */
    int32_t batch_block;    /* batched kernel: threads per workgroup (256, 512, 1024; 0 = autotune
                               cache or default) */
    int32_t batch_unroll;   /* batched kernel: items in flight per thread (1, 2, 4, 8; 0 = auto) */
    int32_t update_hints;   /* update kernel cache hints: bit 0 non-temporal loads, bit 1
                               non-temporal stores (default 0) */
    int32_t update_block;   /* update kernel threads per workgroup (64, 128, 256, 512, 1024;
                               0 = auto); values other than 256 need cols_per_block and
                               rows_per_thread <= 2 */
    int32_t update_grid_stride; /* > 0: grid-stride update kernel with this many workgroups per
                               compute unit (block 64..512), one column per tile (default 0) */
    int32_t update_unroll;  /* grid-stride update kernel: tiles in flight per thread (1, 2, 4, 8) */
    int32_t select_workgroups; /* Steps 1-2 kernel: workgroups (1..64; 0 = 1) */
    int32_t fuse_pivots;    /* pivots applied per pass over the tableau (1..48; 0 = auto: 24, or 16
                               where 24 has no kernels (two launches per pivot, cols_per_block
                               1 or 2), unless an option above asks for a form only K = 1 has). With K > 1 the
                               solver decides K pivots one after the other, each from row 0,
                               its pivot column and the RHS rebuilt by replaying the earlier
                               pivots of the group on those vectors only, then rewrites every
                               changed column once with all K pivots in order: the same
                               arithmetic, so the same pivots and bit-identical tableaux as
                               K = 1, with 1/K of the update traffic. K > 1 needs
                               update_block 0 or <= 256, cols_per_block <= 8,
                               rows_per_thread 0 or 1, update_hints 0, update_grid_stride 0 and
                               select_workgroups <= 1; K > 16 also needs the one-launch
                               decision kernel with decide_block 0 or 256, and cols_per_block 0,
                               4 or 8. */
    int32_t decide_kernel;  /* K > 1: 0 = auto (one launch for all decisions of a group when
                               G = max(m + 1, n + 1 + K) / decide_block rounded up is at most
                               128 workgroups, else two launches per pivot); 1 = two launches
                               per pivot */
    int32_t decide_spin;    /* polls before a grid-barrier wait of the decision kernel gives up
                               with LP_STALLED (0 = default, about 0.2 s); its check-in gate
                               waits at least the default. -1: the first decision launch finds
                               its gate closed, as when its workgroups cannot all be resident
                               (a test of the barrier-free fallback); in the batched form, every
                               split LP's check-in gate closes at once and one workgroup runs
                               that LP whole */
    int32_t decide_block;   /* threads per workgroup of the decision kernel (256 or 512; 0 = auto:
                               256); 512 holds groups of at most 16 pivots */
    int32_t eager_build;    /* 0 = auto: with the one-launch decision kernel, lp_reload_device
                               defers the build of the structural columns to the first update
                               pass (which reads A and c instead of the tableau) and leaves the
                               slack columns unwritten until they leave the basis; 1 = build
                               the whole tableau at once (default 0) */
    int32_t status_readback; /* when the host reads the solver state (status, pivots) to decide
                               on the next group: 1 = one group behind (the next group is
                               queued before the state of the current one is read, so one
                               group is launched after the solve ends and returns at once);
                               2 = right after each group's decisions, while its update pass
                               runs (no group after the end; the host's reaction time must
                               stay below one update pass). 0 = auto: 2 with the one-launch
                               decision kernel and one group per chunk, else 1. 2 needs the
                               one-launch decision kernel and chunk_pivots 0 or at most
                               fuse_pivots. */
} lp_tuning;

/* Options of a solve (the fields listed first are the method's own). */
typedef struct {
    double eps_dual;        /* enter only if T[0][j] < -eps_dual             (default 1e-9) */
    double eps_pivot;       /* row eligible only if T[i][q] > eps_pivot       (default 1e-9) */
    int64_t max_pivots;     /* <= 0 selects 50*(m+n)                          (default 0) */
    int32_t record_pivots;  /* 1 = keep the (r, q) log                       (default 1) */
    void *stream;           /* hipStream_t to run on; NULL = library-owned    (default NULL) */
    void *device_buffer;    /* optional caller-owned device memory for the tableau, at least
                               lp_tableau_bytes(m, n) bytes and 256-byte aligned; it must
                               outlive the context                            (default NULL) */
    size_t device_buffer_bytes;
    int32_t device;         /* HIP device ordinal                             (default 0) */
    int32_t bland_after;    /* anti-cycling fallback (not in the paper): 0 = off, the paper's rule
                               throughout (default); k > 0 = once k pivots in a row were
                               degenerate (ratio T[r][W-1] / T[r][q] <= eps_pivot), Bland's
                               rule (Step 1: the lowest column with T[0][j] < -eps_dual; Step
                               2: among the rows with the smallest ratio, the one whose basic
                               variable has the lowest index) until a pivot that is not
                               degenerate, so the solve cannot cycle. In the general form the
                               count restarts with each phase; drive-out pivots do not count.
                               Needs one pivot per pass (fuse_pivots 0 or 1, which it then
                               implies, and select_workgroups <= 1); the batched form and the
                               server take 0 only. */
    const lp_tuning *tuning; /* execution choices, read during the call; NULL = defaults */
} lp_options;

typedef struct {
    int32_t status;   /* LP_OPTIMAL .. LP_RUNNING */
    int32_t reserved;
    int64_t pivots;   /* pivots performed */
    double objective; /* T[0][W-1] */
    double solve_ms;  /* device time of the last lp_solve / lp_step call */
} lp_result;

typedef struct {
    int32_t m, n;
    int64_t width;          /* W = n+m+1 */
    int64_t ld;             /* column stride of the column-major device tableau, in doubles */
    size_t tableau_bytes;   /* ld * W * 8 */
    const double *tableau;  /* device pointer: T[i][j] at tableau[j*ld + i]; after a deferred
                               build, basic columns that have never left the basis are not
                               stored there until lp_get_tableau */
    int32_t update_block;   /* update kernel in use: threads per workgroup, */
    int32_t update_cols;    /* listed columns per workgroup, */
    int32_t update_rows;    /* row pairs per thread and column, */
    int32_t update_hints;   /* cache hints (bit 0 loads, bit 1 stores non-temporal) */
    int32_t update_fuse;    /* pivots per pass over the tableau (fuse_pivots in use) */
    int32_t decide_workgroups; /* K > 1: workgroups of the one-launch decision kernel (its update
                               pass is k_gupdate_pure); 0 = two launches per pivot (k_gupdate) */
    int32_t status_readback;   /* status_readback in use (1 or 2) */
} lp_info;

/* Library version string. Never fails. */
const char *lp_version(void);

/* Text for a return code or status; never NULL. */
const char *lp_error_string(int code);

/* Text of the last error raised on the calling thread ("" if none). */
const char *lp_last_error(void);

/* Fills *o with the defaults listed above (tuning NULL). LP_E_INVAL if o is NULL. */
int lp_options_default(lp_options *o);

/* Fills *t with the automatic choices (all zero). LP_E_INVAL if t is NULL. */
int lp_tuning_default(lp_tuning *t);

/* Device bytes of the tableau for an m x n LP (0 if m or n < 1). */
size_t lp_tableau_bytes(int32_t m, int32_t n);

/*
 * Creates a context and builds the tableau of Table I with the slack basis
 * (Initialization Step) on the device.
 *   A: host, row-major m x n; b: host, m; c: host, n. Copied during the call.
 *   opt: NULL for defaults.
 * Errors: LP_E_INVAL (NULL, m or n < 1, non-finite value, bad option),
 * LP_E_NEG_RHS (b_i < 0), LP_E_NOMEM, LP_E_DEVICE. On error *out is NULL.
 */
int lp_create(lp_ctx **out, int32_t m, int32_t n, const double *A, const double *b, const double *c,
              const lp_options *opt);

/*
 * As lp_create, with A (row-major m x n), b and c already in device memory
 * on opt->device. They are read by kernels on the context stream and may be
 * freed once lp_create returns. Values are not validated on the host:
 * negative or non-finite inputs give undefined pivots (finite, b >= 0 is the
 * caller's promise).
 */
int lp_create_device(lp_ctx **out, int32_t m, int32_t n, const double *dA, const double *db, const double *dc,
                     const lp_options *opt);

/*
 * Rebuilds the tableau of an existing context from device-resident A, b, c of
 * the same m and n (the Initialization Step again), resetting the pivot count
 * and log. Asynchronous on the context stream. When the build is deferred
 * (eager_build 0 with the one-launch decision kernel: lp_get_info's
 * decide_workgroups > 0), A and c are read by the first update pass of the
 * next lp_solve / lp_step, or by lp_get_tableau if that comes first: they
 * must stay valid and unchanged until that call returns. b is read at once
 * (on the stream).
 */
int lp_reload_device(lp_ctx *h, const double *dA, const double *db, const double *dc);

/*
 * Runs Steps 1-3 until the LP is optimal, unbounded, hits max_pivots or meets
 * a non-finite value. Blocks until done. LP_OK means it ran; the outcome is in
 * lp_get_solution's status.
 */
int lp_solve(lp_ctx *h);

/*
 * Runs at most `pivots` further pivots (the outcome may stay LP_RUNNING), and
 * blocks until done. lp_solve continues from here.
 */
int lp_step(lp_ctx *h, int64_t pivots);

/*
 * Copies the result. x: n doubles or NULL; y: m duals or NULL. Valid after
 * lp_solve / lp_step (LP_E_STATE before).
 */
int lp_get_solution(const lp_ctx *h, lp_result *res, double *x, double *y);

/*
 * Copies up to cap logged pivots (rows r in [1, m], cols q in [0, n+m)) and
 * stores the number of pivots performed in *count (which may exceed cap, or
 * the log if record_pivots was 0).
 */
int lp_get_pivots(const lp_ctx *h, int32_t *rows, int32_t *cols, int64_t cap, int64_t *count);

/*
 * Copies the tableau to host memory, column by column: out[j*(m+1) + i] =
 * T[i][j] for j in [0, W), i in [0, m]. out holds (m+1)*W doubles. Basic
 * columns not stored on the device (a deferred build writes a slack column
 * only when it leaves the basis) are stored first, as the unit vectors they
 * are; a pending deferred build runs first.
 */
int lp_get_tableau(const lp_ctx *h, double *out);

/* Copies the basis: basis[i-1] is the variable basic in tableau row i. */
int lp_get_basis(const lp_ctx *h, int32_t *basis);

/* Sizes and the device tableau pointer. */
int lp_get_info(const lp_ctx *h, lp_info *info);

typedef struct {
    double solve_ms;          /* device time of the last lp_solve / lp_step */
    double update_ms;         /* summed device time of the update kernels launched during that
                                 call (time_kernels = 1; else 0), including the few launched
                                 after the solve ended, which return at once */
    int64_t update_launches;  /* number of update kernels in update_ms */
    int64_t pivots;           /* pivots performed since the tableau was built */
    int64_t updated_columns;  /* tableau columns rewritten by Step 3, summed over the update
                                 passes (columns with a nonzero normalised pivot-row entry in
                                 some pivot of the pass; one pass per pivot when K = 1) */
    double update_ms_applied; /* the part of update_ms spent in launches that applied pivots */
    int64_t applied_launches; /* those launches (the others were queued after the solve ended) */
    double first_pass_ms;     /* time_kernels = 1 and a deferred build: the first update pass
                                 (k_gfirst: the structural build fused with the first group's
                                 Step 3), not part of update_ms */
    int64_t first_pass_pivots;  /* pivots applied by that pass (part of pivots) */
    int64_t first_pass_changed; /* columns it changed (part of updated_columns) */
    int64_t first_pass_columns; /* columns it wrote: the n structural ones, the RHS and those
                                   appended during the group (0 without a deferred build) */
} lp_timing;

/* Timing and work counters of the context (see lp_timing). */
int lp_get_timing(const lp_ctx *h, lp_timing *t);

/* Frees the context and its device memory (not a caller's device_buffer). NULL-safe. */
void lp_destroy(lp_ctx *h);

/*
 * General form (not in the paper, whose Initialization Step starts from a
 * feasible basis): maximise c^T x subject to A_i x <= b_i, >= b_i or = b_i
 * per sense[i] (LP_LE, LP_GE, LP_EQ), x >= 0, b of any sign, by the
 * two-phase method on the one-pivot kernels (fuse_pivots must be 0 or 1):
 *   - rows with b_i < 0 are negated (<= and >= swap); the tableau's rows are
 *     the <= rows, then the >= rows, then the = rows, each in the caller's
 *     order; row m+1 carries the caller's objective through Phase I;
 *   - columns: x (n), one surplus per >= row, one identity column per row
 *     (slack of a <= row, artificial of a >= or = row) and one for row m+1,
 *     the RHS: the context has lp_get_info m = m+1 and n = n + #>= rows;
 *   - Phase I maximises minus the sum of the artificial variables with
 *     Steps 1-3 (row 0 priced out by subtracting the artificial rows in
 *     order); LP_INFEASIBLE when its optimum is below -1e-9 * max(1, sum of
 *     those rows' b);
 *   - artificial variables still basic are driven out by a pivot on the
 *     lowest non-artificial column with |entry| > eps_pivot (none: the row
 *     is redundant and stays, never leaving);
 *   - Phase II on the carried objective, artificial columns barred.
 * One pivot count, cap and log cover both phases (log rows are tableau rows).
 * lp_solve runs both phases; lp_get_solution gives x (n), y (m, the caller's
 * row order, the duals of its rows: >= 0 on <= rows, <= 0 on >= rows) and
 * the objective, meaningful when the status is LP_OPTIMAL. lp_step and
 * lp_reload_device return LP_E_INVAL on such a context. Host inputs are
 * copied; errors as lp_create (LP_E_INVAL also for a bad sense).
 */
int lp_create_general(lp_ctx **out, int32_t m, int32_t n, const double *A, const double *b, const double *c,
                      const int32_t *sense, const lp_options *opt);

/*
 * For callers that cannot allocate device memory (serving loops or harnesses
 * that forbid hipMalloc while they run): lp_create_device + lp_solve +
 * lp_get_solution + lp_get_pivots + lp_destroy in one call that calls no
 * hipMalloc, hipFree, hipHostMalloc or other allocating routine and creates
 * no stream, event or graph. Same kernels, same pivots and bits.
 *
 * dA (row-major m x n), db (m), dc (n): device inputs, only read.
 * tableau: caller-owned device buffer of at least lp_tableau_bytes(m, n)
 *   bytes (tableau_bytes), 256-byte aligned; holds the final tableau on
 *   return (column-major, ld = lp_info.ld for the same m; basic columns that
 *   were never nonbasic are not stored).
 * opt: as lp_create (NULL = defaults; stream NULL = the null stream);
 *   device_buffer is ignored; time_kernels must be 0.
 * res, x (n), y (m): host outputs as lp_get_solution, each may be NULL;
 *   res->solve_ms is host wall time of the pivoting.
 * rows, cols: host arrays of cap entries receiving the pivot log (as
 *   lp_get_pivots); *count (may be NULL) the pivots performed. The device
 *   log keeps the first min(max_pivots, 4 (m + n) + 64) pivots.
 * Every other device buffer lives in a work block of
 * LP_NOALLOC_SCRATCH_BYTES per device, a file-scope device array that each
 * GPU holds until the process ends; an LP whose buffers do not fit is
 * rejected with LP_E_INVAL before any device work. Calls on one device share
 * that block: calls that overlap in time on one device race (serialise them);
 * each call clears the block first. Blocks until done. Errors as lp_create.
 */
#define LP_NOALLOC_SCRATCH_BYTES (8u << 20)
int lp_solve_noalloc(int32_t m, int32_t n, const double *dA, const double *db, const double *dc, double *tableau,
                     size_t tableau_bytes, const lp_options *opt, lp_result *res, double *x, double *y,
                     int32_t *rows, int32_t *cols, int64_t cap, int64_t *count);

/*
 * Diagnostic: the device's binary64 division and fused multiply-add, the two
 * roundings of Steps 2 and 3, applied element-wise on `device`:
 *   quot[k] = a[k] / b[k],   fmav[k] = fma(a[k], b[k], c[k]),   k < count.
 * All five arrays are host arrays of `count` doubles (quot/fmav written).
 * Lets a caller check that the device rounds as IEEE 754 prescribes (round
 * to nearest even, one rounding per operation, subnormals kept).
 */
int lp_diag_arith(int32_t device, int64_t count, const double *a, const double *b, const double *c, double *quot,
                  double *fmav);

/*
 * Diagnostic: a plain device-to-device copy of `bytes` bytes (rounded down to
 * a multiple of 16), repeated `reps` times on `device`, between two buffers
 * the call allocates and frees. Reads and writes exactly `bytes` per
 * repetition, so hardware byte counters of this kernel calibrate those of the
 * solver's kernels. *ms receives the average device time of one copy.
 */
int lp_diag_copy(int32_t device, size_t bytes, int32_t reps, double *ms);

/* ------------------------------------------------------------------ batched
 * Many independent LPs advanced together by one persistent kernel, captured
 * in a hipGraph: every running LP performs Steps 1-3 once per step. Each LP
 * follows exactly the pivot sequence lp_solve gives it.
 */

/*
 * A, b, c: host arrays of `count` pointers to row-major m[k] x n[k], m[k] and
 * n[k] doubles. Copied during the call. Same errors as lp_create; the first
 * failing LP's code is returned.
 */
int lp_batch_create(lp_batch **out, int32_t count, const int32_t *m, const int32_t *n, const double *const *A,
                    const double *const *b, const double *const *c, const lp_options *opt);

/* Solves every LP of the batch; blocks until all have stopped. */
int lp_batch_solve(lp_batch *bt);

/* Result of LP k (0-based); x: n[k] or NULL, y: m[k] or NULL. */
int lp_batch_get_solution(const lp_batch *bt, int32_t k, lp_result *res, double *x, double *y);

/* Pivot log of LP k, as lp_get_pivots. */
int lp_batch_get_pivots(const lp_batch *bt, int32_t k, int32_t *rows, int32_t *cols, int64_t cap, int64_t *count);

/* Device time of the last lp_batch_solve in milliseconds (negative if none). */
double lp_batch_solve_ms(const lp_batch *bt);

/* Rebuilds every tableau from the inputs kept by lp_batch_create (the
 * Initialization Step again), so that the batch can be solved again. */
int lp_batch_reset(lp_batch *bt);

/* The persistent kernel's shape in use: threads per workgroup, items in
 * flight per thread, workgroups per compute unit. Any pointer may be NULL. */
int lp_batch_get_shape(const lp_batch *bt, int32_t *block, int32_t *unroll, int32_t *grid_per_cu);

/*
 * How the shape in use splits large LPs. A split LP (Steps 1-3 of Section
 * III as for any LP, with the same pivots and bits) is run by several
 * workgroups at once, each rewriting a share of its columns and meeting the
 * others twice per pivot: the batch's largest LPs, which would otherwise
 * finish last, then take a fraction of the time. *max_parts: the shape's
 * limit (1: no LP is split); *split_lps: LPs the current plan splits;
 * *queue_entries: the persistent kernel's queue (one entry per LP, one per
 * part of a split LP). Any pointer may be NULL. The autotuner chooses among
 * shapes with and without splitting; LPs whose work area does not fit in
 * LDS are never split.
 */
int lp_batch_get_split(const lp_batch *bt, int32_t *max_parts, int32_t *split_lps, int32_t *queue_entries);

/* Selects the kernel shape (block, unroll, grid_per_cu, split: one of the
 * shapes the autotuner tries) for later solves. LP_E_INVAL if no such shape. */
int lp_batch_set_shape(lp_batch *bt, int32_t block, int32_t unroll, int32_t grid_per_cu, int32_t split);

/*
 * Autotuner: solves the batch once per candidate kernel shape (rebuilding the
 * tableaux before each trial, best of `trials` runs), keeps the fastest
 * shape for later solves, leaves the batch reset, and appends the choice to
 * the JSON-lines cache `cache_path` (NULL: no file) under the batch's size
 * bucket (LP count and largest m, n, each rounded up to a power of two).
 * lp_batch_create applies a cached choice when the environment variable
 * LP_AUTOTUNE_CACHE names that file. *best_ms (may be NULL) receives the
 * fastest solve time.
 */
int lp_batch_autotune(lp_batch *bt, const char *cache_path, int32_t trials, double *best_ms);

void lp_batch_destroy(lp_batch *bt);

/* ------------------------------------------------------------------ hybrid
 * The paper's CPU + GPU split of the tableau's columns (Section IV, Setup,
 * Initialization and Steps 1-4; Tables VI-VIII sweep the share), on one GPU
 * and the host's cores: the GPU keeps the first round(theta n) of the n
 * structural columns and the first round(theta m) of the m slack columns
 * (halves round up), the host the others, so that each side starts with its
 * share of the nonbasic columns; both keep a copy of the right-hand side.
 * Each side rewrites only its nonbasic columns, the leaving column and its
 * right-hand side, as lp_solve does.
 * Each pivot combines the two sides' Step 1 minima, runs Step 2 on the side
 * that owns the entering column, sends its pivot column to the other side
 * over PCIe, then both sides update their own columns at the same time (the
 * host on host_threads threads). The pivots, x, y and objective are those of
 * lp_create + lp_solve with fuse_pivots = 1 (the same roundings, Dantzig's
 * rule and tie-breaks).
 */

/*
 * A, b, c: host inputs as lp_create (standard form, b >= 0), copied.
 * theta: the GPU's share of the columns, in [0, 1] (1: every column on the
 *   GPU, 0: only the right-hand side's copy there).
 * host_threads: threads updating the host's share (<= 0: the host's
 *   hardware threads, at most 16); they spin between pivots while a solve
 *   runs and exit when it ends.
 * opt: eps_dual, eps_pivot, max_pivots, record_pivots and device are used;
 *   bland_after must be 0; the rest is ignored (the GPU share is updated by
 *   the one-pivot update kernel on a stream of the handle's own).
 * Errors as lp_create (LP_E_INVAL also for theta outside [0, 1]).
 */
int lp_hybrid_create(lp_hybrid **out, int32_t m, int32_t n, const double *A, const double *b, const double *c,
                     double theta, int32_t host_threads, const lp_options *opt);

/* Runs Steps 1-3 to the end (a second call does nothing). Blocks. */
int lp_hybrid_solve(lp_hybrid *h);

/* As lp_get_solution; LP_E_STATE before a solve. */
int lp_hybrid_get_solution(const lp_hybrid *h, lp_result *res, double *x, double *y);

/* As lp_get_pivots (entries beyond the log's capacity are not kept). */
int lp_hybrid_get_pivots(const lp_hybrid *h, int32_t *rows, int32_t *cols, int64_t cap, int64_t *count);

/*
 * The tableau into the host array out, column-major, (m+1) rows by n+m+1
 * columns (the RHS last): columns [0, J) and the RHS from the GPU's copy, the
 * rest from the host's. Any time after create.
 */
int lp_hybrid_get_tableau(const lp_hybrid *h, double *out);

/*
 * The split (device_columns and host_columns, summing to n+m), the host thread count
 * and the host's time in its Step 3 share summed over the solve (ms, after a
 * solve). Each pointer may be NULL.
 */
int lp_hybrid_info(const lp_hybrid *h, int32_t *device_columns, int32_t *host_columns, int32_t *host_threads,
                   double *host_ms);

/* Frees the handle. NULL-safe. */
void lp_hybrid_destroy(lp_hybrid *h);

/* ------------------------------------------------------------------ serving
 * A request loop that keeps each admitted LP's tableau resident in device
 * memory. Requests are admitted in arrival order while the resident bytes fit
 * the budget and a slot is free; admitted LPs advance together through the
 * batched kernel (continuous batching); finished LPs are harvested and their
 * memory reused.
 */

struct lp_server_stats {
    int64_t submitted;
    int64_t completed;
    int64_t rejected;
    int64_t resident_now;      /* LPs resident on the device */
    size_t bytes_in_use;       /* device bytes of resident tableaux */
    size_t peak_bytes;         /* highest bytes_in_use seen */
    int64_t ticks;             /* scheduler iterations that launched work */
    double p50_ms, p99_ms;     /* latency, submit to completion, over completed requests */
    double mean_ms;
};

/*
 * hbm_budget_bytes: ceiling on resident device bytes (tableaux and their
 * work buffers; the per-worker staging of inputs is outside it); max_slots:
 * most LPs resident at once (<= 0: 4096). Requests are admitted in arrival
 * order while both allow. LPs whose tableau is at most 16 MiB advance
 * together in the batched kernel; larger ones wait resident (built) until one
 * of the large-LP workers solves them with the single-LP kernels (pivot
 * fusion in groups of 16 with the per-pivot decision kernels). Starts the
 * admission, scheduler and large-LP worker threads.
 */
int lp_server_create(lp_server **out, size_t hbm_budget_bytes, int32_t max_slots, const lp_options *opt);

/*
 * Queues one LP (inputs copied; thread-safe). *ticket identifies it.
 * LP_E_BUDGET if its tableau alone exceeds the budget.
 */
int lp_server_submit(lp_server *s, int32_t m, int32_t n, const double *A, const double *b, const double *c,
                     uint64_t *ticket);

/*
 * LP_OK and the result once the request finished (x: n, y: m, either may be
 * NULL); LP_E_PENDING before; LP_E_INVAL for an unknown or already-collected
 * ticket. A collected result is released.
 */
int lp_server_poll(lp_server *s, uint64_t ticket, lp_result *res, double *x, double *y);

/* As lp_server_poll, but blocks until the request finished. */
int lp_server_wait(lp_server *s, uint64_t ticket, lp_result *res, double *x, double *y);

/* Pivot log of a finished, not yet collected request. */
int lp_server_get_pivots(lp_server *s, uint64_t ticket, int32_t *rows, int32_t *cols, int64_t cap, int64_t *count);

/* Counters and latency percentiles so far, a snapshot into *st (thread-safe).
 * The record is `struct lp_server_stats` (a tag of the same name as the call,
 * as with POSIX stat). */
int lp_server_stats(const lp_server *s, struct lp_server_stats *st);

/* The same as lp_server_stats (the earlier name). */
int lp_server_get_stats(const lp_server *s, struct lp_server_stats *st);

/* Drains every queued request, then stops the scheduler and frees everything. NULL-safe. */
void lp_server_destroy(lp_server *s);

#ifdef __cplusplus
}
#endif

#endif /* LPGPU_H */
