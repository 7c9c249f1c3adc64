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

enum { OR_OPTIMAL = 0, OR_UNBOUNDED = 1, OR_ITER_LIMIT = 2, OR_NUMERICAL = 3, OR_RUNNING = 4, OR_INFEASIBLE = 6 };

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
    /* anti-cycling fallback (oracle_set_bland); see that section */
    int bland_after;  /* 0: off; k > 0: Bland's rule after k consecutive degenerate pivots */
    int degen_run;    /* consecutive degenerate pivots so far */
    /* general form only (oracle_create_general); see that section */
    int general;
    int m_in, n_in;   /* the caller's rows and variables */
    int nprime;       /* structural plus surplus columns */
    int n_le;         /* tableau rows 1..n_le are <= rows (after sign normalisation) */
    int bar;          /* columns >= bar never enter; rows whose basic column is >= bar never leave */
    int phase;        /* 1, 2, or 3 when finished */
    int *perm;        /* tableau row t+1 holds the caller's row perm[t] */
    double *sign;     /* ... multiplied by sign[t] (-1 where b < 0) */
    double feas_scale;
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
    free(o->perm);
    free(o->sign);
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
static int choose_entering_bland(const oracle_lp *o, int limit);
static int choose_leaving_bland(const oracle_lp *o, int q, int bar);
static int use_bland(const oracle_lp *o) { return o->bland_after > 0 && o->degen_run >= o->bland_after; }
static void count_degenerate(oracle_lp *o, int r, int q);

int oracle_step(oracle_lp *o, int64_t steps)
{
    int64_t done = 0;
    while (o->status == OR_RUNNING && (steps < 0 || done < steps)) {
        const int bland = use_bland(o);
        int q = bland ? choose_entering_bland(o, o->n + o->m) : choose_entering(o);
        if (q == -1) { o->status = OR_OPTIMAL; break; }
        if (q == -2) { o->status = OR_NUMERICAL; break; }
        int r = bland ? choose_leaving_bland(o, q, o->n + o->m) : choose_leaving(o, q);
        if (r == -1) { o->status = OR_UNBOUNDED; break; }
        if (r == -2) { o->status = OR_NUMERICAL; break; }
        if (o->pivots >= o->max_pivots) { o->status = OR_ITER_LIMIT; break; }
        count_degenerate(o, r, q);
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

/* ------------------------------------------------------------------------
 * General form: rows A_i x <= b_i, >= b_i or = b_i, any sign of b, x >= 0,
 * by the two-phase method. The paper's Initialization Step starts from a
 * feasible basis (the slack basis of the standard form); this section builds
 * one where there is none, as textbooks do, then runs the paper's Steps 1-3
 * unchanged.
 *
 * Construction (every choice below is a reading; the paper has none):
 *   sign      a row with b_i < 0 is multiplied by -1 (<= and >= swap, =
 *             stays), so every right-hand side is >= 0;
 *   order     tableau rows 1..m are the <= rows, then the >= rows, then the
 *             = rows, each group in the caller's order;
 *   columns   the n structural variables, one surplus variable per >= row
 *             (coefficient -1 in its row; columns n .. n'-1, n' = n + #>=),
 *             then one identity column per row (n'+t-1 for tableau row t:
 *             the slack of a <= row, the artificial variable of a >= or =
 *             row), then one more identity column n'+m for row m+1, then
 *             the right-hand side: W = n' + m + 2 columns;
 *   rows      row m+1 carries the caller's objective through Phase I,
 *             [-c | 0 | e_{m+1} | 0], updated by every pivot like any row;
 *             row 0 is Phase I's objective (maximise minus the sum of the
 *             artificial variables), priced out: start from 1 under each
 *             artificial column and 0 elsewhere, then subtract the
 *             artificial rows one by one in row order;
 *   basis     column n'+t-1 in row t, for t = 1..m+1.
 * Phase I     Steps 1-3 with entering columns j < n'+m (every column but
 *             row m+1's own) and leaving rows whose basic column is < n'+m
 *             (every row but row m+1).
 * Feasibility after an OPTIMAL Phase I: infeasible when the objective
 *             T[0][W-1] (minus the sum of the artificial variables) is below
 *             -1e-9 * max(1, sum of the artificial rows' b), the sum taken
 *             in row order.
 * Drive-out   for t = 1..m in order, where an artificial variable is still
 *             basic: pivot on (t, j) for the lowest column j < n'+n_le (not
 *             artificial) with |T[t][j]| > eps_p; if there is none the row
 *             is redundant and its artificial variable stays basic (at
 *             zero), its row never leaving in Phase II.
 * Phase II    rows 0 and m+1 trade places; Steps 1-3 with entering columns
 *             j < n'+n_le (no artificial column enters) and leaving rows
 *             whose basic column is < n'+n_le.
 * One pivot counter and one log cover both phases and the drive-out.
 * Results     x_j = RHS of the row where j < n is basic; the dual of the
 *             caller's row k, in tableau row t: sign[t] * T[0][n'+t-1];
 *             objective T[0][W-1].
 */

#define OR_FEAS_TOL 1e-9

/* Step 1 over the columns j < bar. -1 optimal, -2 NaN or -inf. */
static int choose_entering_general(const oracle_lp *o)
{
    int q = 0;
    double best = TAB(o, 0, 0);
    for (int j = 0; j < o->bar; ++j) {
        double v = TAB(o, 0, j);
        if (isnan(v)) return -2;
        if (v < best) {
            best = v;
            q = j;
        }
    }
    if (best == -INFINITY) return -2;
    if (best >= -o->eps_d) return -1;
    return q;
}

/* Step 2 over the rows whose basic column is < bar; the non-finite check
 * covers every row 1..m. -1 unbounded, -2 non-finite. */
static int choose_leaving_general(const oracle_lp *o, int q)
{
    const int W = o->W;
    int r = -1;
    double best = 0.0;
    for (int i = 1; i <= o->m; ++i) {
        double a = TAB(o, i, q);
        double rhs = TAB(o, i, W - 1);
        if (!isfinite(a) || isnan(rhs)) return -2;
        if (a > o->eps_p && o->basis[i - 1] < o->bar) {
            double ratio = rhs / a;
            if (r < 0 || ratio < best) {
                best = ratio;
                r = i;
            }
        }
    }
    return r;
}

/* Logs pivot (r, q) and counts it. */
static void log_pivot(oracle_lp *o, int r, int q)
{
    if (o->pivots < o->log_cap) {
        o->log_r[o->pivots] = r;
        o->log_q[o->pivots] = q;
    }
    o->pivots++;
}

/* sense: 0 for <=, 1 for >=, 2 for =. Returns NULL on bad input (m or n < 1,
 * a non-finite value, an unknown sense). */
oracle_lp *oracle_create_general(int m, int n, const double *A, const double *b, const double *c,
                                 const int *sense, double eps_d, double eps_p, int64_t max_pivots,
                                 int64_t log_cap, int nthreads)
{
    if (m < 1 || n < 1 || !A || !b || !c || !sense) return NULL;
    for (int64_t k = 0; k < (int64_t)m * n; ++k)
        if (!isfinite(A[k])) return NULL;
    for (int i = 0; i < m; ++i)
        if (!isfinite(b[i]) || sense[i] < 0 || sense[i] > 2) return NULL;
    for (int j = 0; j < n; ++j)
        if (!isfinite(c[j])) return NULL;

    /* normalised sense of each caller row and the tableau order */
    int *kind = (int *)calloc((size_t)m, sizeof(int));
    if (!kind) return NULL;
    int n_le = 0, n_ge = 0;
    for (int i = 0; i < m; ++i) {
        int k = sense[i];
        if (b[i] < 0.0 && k != 2) k = 1 - k;
        kind[i] = k;
        n_le += k == 0;
        n_ge += k == 1;
    }
    const int np = n + n_ge;
    const int M = m + 1; /* constraint rows and the carried objective row */
    oracle_lp *o = (oracle_lp *)calloc(1, sizeof(oracle_lp));
    if (!o) {
        free(kind);
        return NULL;
    }
    o->m = M;
    o->n = np;
    o->W = np + M + 1;
    o->T = (double *)calloc((size_t)(M + 1) * (size_t)o->W, sizeof(double));
    o->F = (double *)calloc((size_t)M + 1, sizeof(double));
    o->R = (double *)calloc((size_t)o->W, sizeof(double));
    o->basis = (int *)calloc((size_t)M, sizeof(int));
    o->perm = (int *)calloc((size_t)m, sizeof(int));
    o->sign = (double *)calloc((size_t)m, sizeof(double));
    o->log_cap = log_cap > 0 ? log_cap : 0;
    if (o->log_cap) {
        o->log_r = (int *)calloc((size_t)o->log_cap, sizeof(int));
        o->log_q = (int *)calloc((size_t)o->log_cap, sizeof(int));
    }
    if (!o->T || !o->F || !o->R || !o->basis || !o->perm || !o->sign ||
        (o->log_cap && (!o->log_r || !o->log_q))) {
        free(kind);
        oracle_destroy(o);
        return NULL;
    }
    o->eps_d = eps_d;
    o->eps_p = eps_p;
    o->max_pivots = max_pivots;
    o->nthreads = nthreads > 0 ? nthreads : 1;
    o->status = OR_RUNNING;
    o->general = 1;
    o->m_in = m;
    o->n_in = n;
    o->nprime = np;
    o->n_le = n_le;
    o->phase = 1;
    o->bar = np + m;

    int t = 0;
    for (int want = 0; want < 3; ++want)
        for (int i = 0; i < m; ++i)
            if (kind[i] == want) {
                o->perm[t] = i;
                o->sign[t] = b[i] < 0.0 ? -1.0 : 1.0;
                ++t;
            }
    free(kind);

    const int W = o->W;
    int surplus = n;
    for (int t1 = 1; t1 <= m; ++t1) {
        const int k = o->perm[t1 - 1];
        const double s = o->sign[t1 - 1];
        for (int j = 0; j < n; ++j) TAB(o, t1, j) = s == 1.0 ? A[(size_t)k * n + j] : -A[(size_t)k * n + j];
        if (t1 > n_le && t1 <= n_le + n_ge) TAB(o, t1, surplus++) = -1.0;
        TAB(o, t1, np + t1 - 1) = 1.0;
        TAB(o, t1, W - 1) = s == 1.0 ? b[k] : -b[k];
        o->basis[t1 - 1] = np + t1 - 1;
    }
    for (int j = 0; j < n; ++j) TAB(o, M, j) = -c[j];
    TAB(o, M, np + m) = 1.0;
    o->basis[M - 1] = np + m;
    /* Phase I's objective row, priced out */
    for (int j = 0; j < W; ++j) TAB(o, 0, j) = (j >= np + n_le && j < np + m) ? 1.0 : 0.0;
    double scale = 0.0;
    for (int t1 = n_le + 1; t1 <= m; ++t1) {
        for (int j = 0; j < W; ++j) TAB(o, 0, j) = TAB(o, 0, j) - TAB(o, t1, j);
        scale = scale + TAB(o, t1, W - 1);
    }
    o->feas_scale = scale > 1.0 ? scale : 1.0;
    return o;
}

/* Steps 1-3 until the phase ends (or the cap). */
static void run_phase(oracle_lp *o)
{
    o->degen_run = 0; /* each phase starts with the usual rule */
    while (o->status == OR_RUNNING) {
        const int bland = use_bland(o);
        int q = bland ? choose_entering_bland(o, o->bar) : choose_entering_general(o);
        if (q == -1) { o->status = OR_OPTIMAL; break; }
        if (q == -2) { o->status = OR_NUMERICAL; break; }
        int r = bland ? choose_leaving_bland(o, q, o->bar) : choose_leaving_general(o, q);
        if (r == -1) { o->status = OR_UNBOUNDED; break; }
        if (r == -2) { o->status = OR_NUMERICAL; break; }
        if (o->pivots >= o->max_pivots) { o->status = OR_ITER_LIMIT; break; }
        count_degenerate(o, r, q);
        pivot(o, r, q);
        log_pivot(o, r, q);
    }
}

/* Both phases. Returns the final status. */
int oracle_solve_general(oracle_lp *o)
{
    if (!o->general || o->phase != 1) return o->status;
    const int m = o->m_in, np = o->nprime, W = o->W;
    run_phase(o);
    if (o->status != OR_OPTIMAL) {
        o->phase = 3;
        return o->status;
    }
    const double w = TAB(o, 0, W - 1);
    if (isnan(w)) {
        o->status = OR_NUMERICAL;
        o->phase = 3;
        return o->status;
    }
    if (w < -OR_FEAS_TOL * o->feas_scale) {
        o->status = OR_INFEASIBLE;
        o->phase = 3;
        return o->status;
    }
    /* drive the artificial variables still basic out of the basis */
    const int allowed = np + o->n_le;
    for (int t = 1; t <= m; ++t) {
        if (o->basis[t - 1] < allowed) continue;
        int q = -1;
        for (int j = 0; j < allowed; ++j)
            if (fabs(TAB(o, t, j)) > o->eps_p) {
                q = j;
                break;
            }
        if (q < 0) continue; /* redundant row */
        if (o->pivots >= o->max_pivots) {
            o->status = OR_ITER_LIMIT;
            o->phase = 3;
            return o->status;
        }
        pivot(o, t, q);
        log_pivot(o, t, q);
    }
    /* Phase II: the carried objective becomes row 0 */
    for (int j = 0; j < W; ++j) {
        const double v = TAB(o, 0, j);
        TAB(o, 0, j) = TAB(o, m + 1, j);
        TAB(o, m + 1, j) = v;
    }
    o->bar = allowed;
    o->phase = 2;
    o->status = OR_RUNNING;
    run_phase(o);
    o->phase = 3;
    return o->status;
}

/* x (n_in), y (m_in, the caller's row order) and the objective. */
void oracle_extract_general(const oracle_lp *o, double *x, double *y, double *objective)
{
    const int m = o->m_in, np = o->nprime, W = o->W;
    if (x) {
        for (int j = 0; j < o->n_in; ++j) x[j] = 0.0;
        for (int t = 1; t <= m; ++t)
            if (o->basis[t - 1] < o->n_in) x[o->basis[t - 1]] = TAB(o, t, W - 1);
    }
    if (y)
        for (int t = 1; t <= m; ++t) {
            const double v = TAB(o, 0, np + t - 1);
            y[o->perm[t - 1]] = o->sign[t - 1] == 1.0 ? v : -v;
        }
    if (objective) *objective = TAB(o, 0, W - 1);
}

/* The layout of a general-form tableau: n', n_le, the phase reached, and the
 * caller's row of each tableau row with its sign. */
void oracle_general_layout(const oracle_lp *o, int *nprime, int *n_le, int *phase, int *perm, double *sign)
{
    if (nprime) *nprime = o->nprime;
    if (n_le) *n_le = o->n_le;
    if (phase) *phase = o->phase;
    if (perm) memcpy(perm, o->perm, (size_t)o->m_in * sizeof(int));
    if (sign) memcpy(sign, o->sign, (size_t)o->m_in * sizeof(double));
}

/* ------------------------------------------------------------------------
 * Anti-cycling fallback. The paper's rule (most negative row-0 entry, lowest
 * index on ties; minimum ratio, lowest row on ties) can cycle on degenerate
 * LPs; the iteration cap then ends the solve. With bland_after = k > 0 the
 * solve switches to Bland's rule once k pivots in a row were degenerate, and
 * back to the usual rule after the first pivot that is not:
 *   degenerate   a pivot whose ratio T[r][W-1] / T[r][q] (the step length,
 *                the same division as Step 2) is at most eps_p: a step the
 *                pivot tolerance does not tell from no step (the objective
 *                does not improve, up to round-off);
 *   Bland, Step 1  the lowest column j (below the bar) with
 *                T[0][j] < -eps_d; the non-finite checks and the optimality
 *                test are those of Step 1;
 *   Bland, Step 2  among the eligible rows with the smallest ratio, the one
 *                whose basic variable has the lowest index; the non-finite
 *                checks are those of Step 2.
 * Bland's rule cannot cycle, and every stretch of degenerate pivots longer
 * than k runs under it, so the solve terminates. In the general form the
 * count starts at 0 in each phase and the drive-out pivots leave it alone.
 */

/* Step 1 under Bland's rule over the columns j < limit. */
static int choose_entering_bland(const oracle_lp *o, int limit)
{
    int q = -1;
    double best = INFINITY;
    for (int j = 0; j < limit; ++j) {
        double v = TAB(o, 0, j);
        if (isnan(v)) return -2;
        if (v < best) best = v;
        if (q < 0 && v < -o->eps_d) q = j;
    }
    if (best == -INFINITY) return -2;
    return q; /* -1: optimal */
}

/* Step 2 under Bland's rule; rows whose basic column is >= bar never leave. */
static int choose_leaving_bland(const oracle_lp *o, int q, int bar)
{
    const int W = o->W;
    int r = -1;
    double best = 0.0;
    for (int i = 1; i <= o->m; ++i) {
        double a = TAB(o, i, q);
        double rhs = TAB(o, i, W - 1);
        if (!isfinite(a) || isnan(rhs)) return -2;
        if (a > o->eps_p && o->basis[i - 1] < bar) {
            double ratio = rhs / a;
            if (r < 0 || ratio < best || (ratio == best && o->basis[i - 1] < o->basis[r - 1])) {
                best = ratio;
                r = i;
            }
        }
    }
    return r;
}

/* Before pivot (r, q): counts it as degenerate or resets the count. */
static void count_degenerate(oracle_lp *o, int r, int q)
{
    const double theta = TAB(o, r, o->W - 1) / TAB(o, r, q);
    o->degen_run = theta <= o->eps_p ? o->degen_run + 1 : 0;
}

/* Sets k (0 = off); call before the first step. */
void oracle_set_bland(oracle_lp *o, int bland_after)
{
    o->bland_after = bland_after > 0 ? bland_after : 0;
    o->degen_run = 0;
}
