/*
 * Plain CPU reference of the full-tableau primal simplex method.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU solver never
 * calls it, links it or shares code with it.
 *
 * What it computes (Mamalis & Perlitis, Section III):
 *   Problem      max c^T x  s.t.  A x <= b,  x >= 0,  b >= 0  (standard form).
 *   Tableau      Table I, row-major, (m+1) rows by W = n+m+1 columns:
 *                  row 0      = [ -c_1 .. -c_n | 0 .. 0 | 0   ]
 *                  row i>=1   = [  A_i1 .. A_in | e_i    | b_i ]
 *                The z column of Table I is left out: it is the unit vector
 *                e_0 before and after every pivot, because the pivot row is
 *                never row 0.
 *   Initialization Step  the slack basis; basis[i-1] = n+i-1.
 *   Step 1 (entering)    q = the column with the most negative row-0 entry
 *                        over j in [0, n+m); ties go to the lowest j. If that
 *                        entry is >= -eps_d the tableau is optimal.
 *   Step 2 (leaving)     over rows i in [1, m] with T[i][q] > eps_p, the
 *                        smallest ratio T[i][W-1] / T[i][q]; ties go to the
 *                        lowest i. No such row: unbounded.
 *   Step 3 (pivoting)    p = T[r][q]; F = column q before the update;
 *                        R_j = T[r][j] / p for every j;
 *                        T[i][j] = fma(-F_i, R_j, T[i][j]) for i != r;
 *                        T[r][j] = R_j; basis[r-1] = q.
 *   Iterate/Finalization repeat Steps 1-3 until optimal or unbounded. An
 *                        iteration cap (checked after Step 2, before the
 *                        pivot) stops with ITER_LIMIT.
 *   Non-finite values    the paper does not discuss them. Read here as: Step 1
 *                        stops with NUMERICAL when row 0 holds a NaN or its
 *                        smallest entry is -inf; Step 2 stops with NUMERICAL
 *                        when, in some row 1..m (eligible or not), the
 *                        entering column holds a value that is not finite or
 *                        the RHS holds a NaN. A ratio that overflows is an
 *                        ordinary infinite ratio.
 *
 * Arithmetic: IEEE binary64, division for R and the ratios, one fused
 * multiply-add per updated entry. Build with -ffp-contract=off and no
 * fast-math so that nothing else is fused or reordered.
 *
 * The only parallelism is an OpenMP loop over the rows of Step 3; every row is
 * updated by the same formula, so the result does not depend on the number of
 * threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_OPTIMAL = 0, OR_UNBOUNDED = 1, OR_ITER_LIMIT = 2, OR_NUMERICAL = 3, OR_RUNNING = 4 };

typedef struct {
    int m, n, W;
    double *T;        /* (m+1) x W, row-major */
    double *F;        /* m+1: pivot column snapshot */
    double *R;        /* W: normalised pivot row */
    int *basis;       /* m */
    double eps_d, eps_p;
    int64_t max_pivots;
    int64_t pivots;
    int status;
    int *log_r, *log_q;
    int64_t log_cap;
    int nthreads;
} oracle_lp;

#define TAB(o, i, j) ((o)->T[(size_t)(i) * (size_t)(o)->W + (size_t)(j)])

void oracle_destroy(oracle_lp *o)
{
    if (!o) return;
    free(o->T);
    free(o->F);
    free(o->R);
    free(o->basis);
    free(o->log_r);
    free(o->log_q);
    free(o);
}

/* Initialization Step: Table I with the slack basis. Returns NULL on bad input
 * (m or n < 1, a non-finite value, or some b_i < 0). */
oracle_lp *oracle_create(int m, int n, const double *A, const double *b, const double *c,
                         double eps_d, double eps_p, int64_t max_pivots, int64_t log_cap,
                         int nthreads)
{
    if (m < 1 || n < 1 || !A || !b || !c) return NULL;
    for (int64_t k = 0; k < (int64_t)m * n; ++k)
        if (!isfinite(A[k])) return NULL;
    for (int i = 0; i < m; ++i)
        if (!isfinite(b[i]) || b[i] < 0.0) return NULL;
    for (int j = 0; j < n; ++j)
        if (!isfinite(c[j])) return NULL;

    oracle_lp *o = (oracle_lp *)calloc(1, sizeof(oracle_lp));
    if (!o) return NULL;
    o->m = m;
    o->n = n;
    o->W = n + m + 1;
    o->T = (double *)calloc((size_t)(m + 1) * (size_t)o->W, sizeof(double));
    o->F = (double *)calloc((size_t)m + 1, sizeof(double));
    o->R = (double *)calloc((size_t)o->W, sizeof(double));
    o->basis = (int *)calloc((size_t)m, sizeof(int));
    o->log_cap = log_cap > 0 ? log_cap : 0;
    if (o->log_cap) {
        o->log_r = (int *)calloc((size_t)o->log_cap, sizeof(int));
        o->log_q = (int *)calloc((size_t)o->log_cap, sizeof(int));
    }
    if (!o->T || !o->F || !o->R || !o->basis || (o->log_cap && (!o->log_r || !o->log_q))) {
        oracle_destroy(o);
        return NULL;
    }
    o->eps_d = eps_d;
    o->eps_p = eps_p;
    o->max_pivots = max_pivots;
    o->nthreads = nthreads > 0 ? nthreads : 1;
    o->status = OR_RUNNING;

    const int W = o->W;
    for (int j = 0; j < n; ++j) TAB(o, 0, j) = -c[j];
    for (int i = 1; i <= m; ++i) {
        for (int j = 0; j < n; ++j) TAB(o, i, j) = A[(size_t)(i - 1) * n + j];
        TAB(o, i, n + i - 1) = 1.0;
        TAB(o, i, W - 1) = b[i - 1];
        o->basis[i - 1] = n + i - 1;
    }
    return o;
}

/* Step 1. Returns the entering column, -1 when optimal, -2 when row 0 holds a
 * NaN or its smallest entry is -inf. */
static int choose_entering(const oracle_lp *o)
{
    int q = 0;
    double best = TAB(o, 0, 0);
    for (int j = 0; j < o->n + o->m; ++j) {
        double v = TAB(o, 0, j);
        if (isnan(v)) return -2;
        if (v < best) { /* strict: an equal value later keeps the lower index */
            best = v;
            q = j;
        }
    }
    if (best == -INFINITY) return -2;
    if (best >= -o->eps_d) return -1;
    return q;
}

/* Step 2. Returns the leaving row in [1, m], -1 when unbounded, -2 when some
 * row holds a non-finite entering-column value or a NaN right-hand side. */
static int choose_leaving(const oracle_lp *o, int q)
{
    const int W = o->W;
    int r = -1;
    double best = 0.0;
    for (int i = 1; i <= o->m; ++i) {
        double a = TAB(o, i, q);
        double rhs = TAB(o, i, W - 1);
        if (!isfinite(a) || isnan(rhs)) return -2;
        if (a > o->eps_p) {
            double ratio = rhs / a; /* finite a > 0 and a non-NaN rhs: never NaN */
            if (r < 0 || ratio < best) {
                best = ratio;
                r = i;
            }
        }
    }
    return r;
}

/* Step 3 on pivot (r, q). */
static void pivot(oracle_lp *o, int r, int q)
{
    const int m = o->m, W = o->W;
    const double p = TAB(o, r, q);
    for (int i = 0; i <= m; ++i) o->F[i] = TAB(o, i, q);
    for (int j = 0; j < W; ++j) o->R[j] = TAB(o, r, j) / p;

    const double *R = o->R;
    const double *F = o->F;
#pragma omp parallel for schedule(static) num_threads(o->nthreads)
    for (int i = 0; i <= m; ++i) {
        double *row = &TAB(o, i, 0);
        if (i == r) {
            for (int j = 0; j < W; ++j) row[j] = R[j];
        } else {
            const double mf = -F[i];
            for (int j = 0; j < W; ++j) row[j] = fma(mf, R[j], row[j]);
        }
    }
    o->basis[r - 1] = q;
}

/* Runs up to `steps` pivots (all remaining when steps < 0). Returns the status;
 * OR_RUNNING means the step budget ran out with work left. */
int oracle_step(oracle_lp *o, int64_t steps)
{
    int64_t done = 0;
    while (o->status == OR_RUNNING && (steps < 0 || done < steps)) {
        int q = choose_entering(o);
        if (q == -1) { o->status = OR_OPTIMAL; break; }
        if (q == -2) { o->status = OR_NUMERICAL; break; }
        int r = choose_leaving(o, q);
        if (r == -1) { o->status = OR_UNBOUNDED; break; }
        if (r == -2) { o->status = OR_NUMERICAL; break; }
        if (o->pivots >= o->max_pivots) { o->status = OR_ITER_LIMIT; break; }
        pivot(o, r, q);
        if (o->pivots < o->log_cap) {
            o->log_r[o->pivots] = r;
            o->log_q[o->pivots] = q;
        }
        o->pivots++;
        done++;
    }
    return o->status;
}

int oracle_status(const oracle_lp *o) { return o->status; }
int64_t oracle_pivots(const oracle_lp *o) { return o->pivots; }
int oracle_width(const oracle_lp *o) { return o->W; }

/* Copies the tableau, (m+1) x W row-major. */
void oracle_get_tableau(const oracle_lp *o, double *out)
{
    memcpy(out, o->T, (size_t)(o->m + 1) * (size_t)o->W * sizeof(double));
}

void oracle_get_basis(const oracle_lp *o, int *out) { memcpy(out, o->basis, (size_t)o->m * sizeof(int)); }

/* Copies up to cap logged pivots; returns how many were copied. */
int64_t oracle_get_log(const oracle_lp *o, int *rows, int *cols, int64_t cap)
{
    int64_t k = o->pivots < o->log_cap ? o->pivots : o->log_cap;
    if (k > cap) k = cap;
    if (k > 0) {
        memcpy(rows, o->log_r, (size_t)k * sizeof(int));
        memcpy(cols, o->log_q, (size_t)k * sizeof(int));
    }
    return k;
}

/* Finalization: x_j = RHS of the row where j is basic (0 if nonbasic),
 * y_i = row-0 entry of slack column n+i-1, objective = row-0 RHS. */
void oracle_extract(const oracle_lp *o, double *x, double *y, double *objective)
{
    const int m = o->m, n = o->n, W = o->W;
    if (x) {
        for (int j = 0; j < n; ++j) x[j] = 0.0;
        for (int i = 1; i <= m; ++i)
            if (o->basis[i - 1] < n) x[o->basis[i - 1]] = TAB(o, i, W - 1);
    }
    if (y)
        for (int i = 1; i <= m; ++i) y[i - 1] = TAB(o, 0, n + i - 1);
    if (objective) *objective = TAB(o, 0, W - 1);
}
