/*
 * psl_oracle.c -- sequential CPU reference presolver (TEST INFRASTRUCTURE).
 *
 * Not part of the product: only tests, the smoke check and the benchmark's
 * CPU-baseline leg load this. It is deliberately plain and slow. Build with
 * -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 *
 * What it computes follows the paper (Cederberg & Boyd, "GPU-Accelerated
 * Presolving for Linear Programming"):
 *   - LP form: eq. (1), section 2.1.
 *   - Reductions with a postsolve record each: section 2.1, "Reductions" and
 *     "Postsolver"; fixing stores only index and value.
 *   - Bound tightening from min/max activities, repeated in rounds until a
 *     round tightens nothing or a round cap is hit: section 3.1, "Bound
 *     tightening" (worked example x1 + 2 x2 <= 4, x >= 0 => x1 <= 4, x2 <= 2).
 *   - Inactive flags instead of physical removal; activities recomputed on
 *     demand; row and column sizes maintained: section 3.2, "Internal data
 *     structures".
 *   - Parallel rows by a two-level hash on pattern and coefficients, verified
 *     against a leader (first equality of the group, else first inequality):
 *     section 3.2, "Parallel rows".
 *   - Emission of a reduced LP of the same form and primal recovery:
 *     section 3.3.
 *   - Optional (off by default): dual fixing from variable locks recounted
 *     on demand (section 3.2, "Internal data structures"; dual explorers,
 *     section 2.1), see dual_fix below.
 *
 * Readings where the paper is silent (they define the round semantics that
 * the GPU library must reproduce bit for bit):
 *   R-Jacobi  every test in a round reads the bounds as they were at the start
 *             of the round; tightenings are combined by max/min (the paper's
 *             in-place atomic updates are order dependent).
 *   R-Sum     every sum of a row (activities, fixed-column constants) and the
 *             objective offset is the canonical pairwise tree: leaves are the
 *             row's CSR positions 0..len-1 padded with +0 to the next power of
 *             two, each node is fl(left + right); terms equal to zero are +0.
 *   R-Bound   implied bounds from residual activities with infinite-bound
 *             counts (formulas in propagate_row below).
 *   R-Tol     tol(s) = feas_tol * max(1, |s|); candidate bound qualifies if it
 *             improves by more than min_improve * max(1, |bound|) (any strict
 *             improvement for a row with one active column).
 *   R-Hash    parallel-row key over the row's active entries (pattern and
 *             coefficients normalised by the first active coefficient), mixed
 *             with the SplitMix64 finaliser (Steele, Lea & Flood 2014);
 *             merged sides are compared after moving the removed columns'
 *             constant contribution out of them (see parallel_rows).
 *   R-Order   records ordered by (round, phase, index, side).
 */
#include "psl_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { RES_REDUCED = 0, RES_UNCHANGED = 1, RES_INFEASIBLE = 2, RES_UNBOUNDED = 3 };

/* record types; fields (unused ints are -1, unused doubles 0):
 *  FIX_COL        j; v = {value, c_j}
 *  EMPTY_COL      j; v = {value, c_j}
 *  EMPTY_ROW      i; v = {activity, lhs, rhs}
 *  REDUNDANT_ROW  i; v = {min activity or -inf, max activity or +inf, lhs, rhs}
 *  SINGLETON_ROW  i, j = the active column; v = {a_ij, lhs, rhs}
 *  BOUND_CHANGE   j, side (0 lower, 1 upper), k = source row;
 *                 v = {old bound, new bound, a_kj}
 *  PARALLEL_ROW   i = removed row, k = leader; v = {lambda, lhs_i, rhs_i}
 *  LEADER_SIDES   i = leader, j = row giving lhs, k = row giving rhs;
 *                 v = {old lhs, old rhs, new lhs, new rhs}
 *  DUAL_FIX       j, side (0 fixed at its lower, 1 at its upper bound);
 *                 v = {value, c_j}
 *  FREE_SINGLETON i = removed row, j = its (implied) free column; side 0:
 *                 c_j = 0, 1: the row went to its lhs, 2: to its rhs;
 *                 v = {a_ij, lhs_i, rhs_i (the sides then), c_j (then)}
 *  PARALLEL_COL   j = merged column, k = its leader; v = {lambda, lb_j, ub_j}
 *  LEADER_BOUNDS  j = leader; v = {old lb, old ub, new lb, new ub}
 *  FORCING_ROW    i; side 0: the min activity reaches rhs (every active
 *                 column at the bound of its min contribution), 1: the max
 *                 activity reaches lhs; v = {that activity, lhs, rhs}
 *  DOUBLETON_ROW  i = the equality row, j = the kept column, k = the
 *                 eliminated one; v = {a_ij, a_ik, b (the row's side moved by
 *                 its removed columns' constant), c_k (then)}
 *  DOMINATED_COL  j, side (0 fixed at its lower, 1 at its upper bound);
 *                 v = {value, c_j}
 */
enum {
    REC_FIX_COL = 1, REC_EMPTY_COL = 2, REC_EMPTY_ROW = 3, REC_REDUNDANT_ROW = 4,
    REC_SINGLETON_ROW = 5, REC_BOUND_CHANGE = 6, REC_PARALLEL_ROW = 7, REC_LEADER_SIDES = 8,
    REC_DUAL_FIX = 9, REC_FREE_SINGLETON = 10, REC_PARALLEL_COL = 11, REC_LEADER_BOUNDS = 12,
    REC_FORCING_ROW = 13, REC_DOUBLETON_ROW = 14, REC_DOMINATED_COL = 15
};

/* classes of the reduced problem's rows and columns (listed, not applied) */
enum { RCLS_OTHER = 0, RCLS_SINGLETON = 1, RCLS_DOUBLETON_EQ = 2, RCLS_DOUBLETON_INEQ = 3 };
enum { CCLS_OTHER = 0, CCLS_SINGLETON_FREE = 1, CCLS_SINGLETON = 2, CCLS_DOUBLETON = 3 };

struct or_handle {
    int32_t m, n;
    int64_t nnz;
    int32_t *rp, *ci;
    double *va;
    double *lhs, *rhs, *lb, *ub, *c, off;
    double *c0;  /* the input costs (c changes when a singleton is substituted) */
    int32_t *ci0; /* the input matrix's entries (doubleton substitutions rewrite */
    double *va0;  /* rows in place; the dual postsolve needs the input's)       */
    uint8_t *col_mod; /* column kept by a doubleton substitution (entries changed) */
    or_settings s;

    uint8_t *row_on, *col_on;
    int32_t *col_len;
    /* per side of each column: -1 the input bound was infinite and is
     * unchanged, r >= 0 it was infinite and every tightening came from row r,
     * -2 otherwise (free column singletons: bounds implied by their row) */
    int32_t *lsrc, *usrc;
    /* the matrix by columns (rows ascending within a column) */
    int32_t *cp, *ri;
    double *cva;

    or_record *rec;
    int64_t nrec, caprec;

    int32_t result, round;
    char err[256];

    /* reduced problem */
    int32_t rm, rn;
    int64_t rnnz;
    double roff;
    int32_t *r_rp, *r_ci, *r_cp, *r_ri, *r_rowmap, *r_colmap;
    double *r_va, *r_cva, *r_lhs, *r_rhs, *r_lb, *r_ub, *r_c;
    uint8_t *r_rcls, *r_ccls;
};

/* ------------------------------------------------------------------------- */
/* small helpers                                                              */
/* ------------------------------------------------------------------------- */

static double pos0(double x) { return x == 0.0 ? 0.0 : x; } /* -0 -> +0 */
static double mx1(double x) { double a = fabs(x); return a > 1.0 ? a : 1.0; }
static double tol_of(const or_settings *s, double x) { return s->feas_tol * mx1(x); }

static void *xcalloc(size_t n, size_t sz) {
    void *p = calloc(n ? n : 1, sz);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

static void push(or_handle *h, int type, int side, int32_t i, int32_t j, int32_t k,
                 double v0, double v1, double v2, double v3) {
    if (h->nrec == h->caprec) {
        h->caprec = h->caprec ? 2 * h->caprec : 1024;
        h->rec = (or_record *)realloc(h->rec, (size_t)h->caprec * sizeof(or_record));
        if (!h->rec) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    }
    or_record *r = &h->rec[h->nrec++];
    memset(r, 0, sizeof *r);
    r->type = (uint8_t)type;
    r->side = (uint8_t)side;
    r->round = (uint16_t)h->round;
    r->i = i; r->j = j; r->k = k;
    r->v[0] = v0; r->v[1] = v1; r->v[2] = v2; r->v[3] = v3;
}

/* ------------------------------------------------------------------------- */
/* canonical pairwise sum (reading R-Sum)                                     */
/* ------------------------------------------------------------------------- */

/* Sum of the aligned block [lo, lo+size) of the padded leaf sequence. */
static double pw_block(const double *x, int64_t len, int64_t lo, int64_t size) {
    if (lo >= len) return 0.0;            /* an all-padding block sums to +0 */
    if (size == 1) return x[lo];
    int64_t h = size / 2;
    double left = pw_block(x, len, lo, h);
    double right = pw_block(x, len, lo + h, h);
    return left + right;
}

double or_pairwise_sum(const double *x, int64_t len) {
    if (len <= 0) return 0.0;
    int64_t p = 1;
    while (p < len) p <<= 1;
    return pw_block(x, len, 0, p);
}

/* ------------------------------------------------------------------------- */
/* parallel-row key (reading R-Hash)                                          */
/* ------------------------------------------------------------------------- */

/* SplitMix64 output function for state x (Steele, Lea & Flood 2014). */
static uint64_t splitmix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* keep sign, exponent and the top 32 mantissa bits, rounded to nearest */
static uint64_t quantize(double v) {
    uint64_t b;
    memcpy(&b, &v, 8);
    uint64_t sign = b >> 63;
    uint64_t mag = b & 0x7FFFFFFFFFFFFFFFULL;
    uint64_t q = (mag + (1ULL << 19)) >> 20;
    return q | (sign << 63);
}

uint64_t or_row_key(const int32_t *cols, const double *vals, int64_t len) {
    /* level 1: sparsity pattern; level 2: normalised coefficients */
    uint64_t h1 = (uint64_t)len;
    uint64_t h2 = 0;
    for (int64_t k = 0; k < len; ++k) {
        uint64_t cj = splitmix((uint64_t)(uint32_t)cols[k]);
        double v = vals[k] / vals[0];
        h1 += cj;
        h2 += splitmix(cj ^ quantize(v));
    }
    return (splitmix(h1) ^ h2) | 1ULL;
}

/* ------------------------------------------------------------------------- */
/* validation and ingest                                                      */
/* ------------------------------------------------------------------------- */

static int fail(or_handle *h, const char *msg) {
    snprintf(h->err, sizeof h->err, "%s", msg);
    return 1;
}

static double canon_inf(double v, double inf_value) {
    if (v >= inf_value) return INFINITY;
    if (v <= -inf_value) return -INFINITY;
    return pos0(v);
}

static int validate_and_copy(or_handle *h, const or_lp *lp, const or_settings *s) {
    if (s->max_rounds < 1 || s->max_outer < 1 ||
        (int64_t)s->max_outer * (s->max_rounds + 1) + 1 > 65535)
        return fail(h, "invalid round limits");
    if (!(s->feas_tol >= 0) || !(s->fix_tol >= 0) || !(s->min_improve >= 0) ||
        !(s->par_tol >= 0) || !(s->inf_value > 0) || !(s->coef_tol >= 0))
        return fail(h, "invalid tolerance");
    if (s->enable_dual_fix != 0 && s->enable_dual_fix != 1) return fail(h, "invalid dual-fix switch");
    if (s->enable_free_singletons != 0 && s->enable_free_singletons != 1)
        return fail(h, "invalid free-singleton switch");
    if (s->enable_forcing_rows != 0 && s->enable_forcing_rows != 1) return fail(h, "invalid settings");
    if (s->enable_doubletons != 0 && s->enable_doubletons != 1) return fail(h, "invalid settings");
    if (s->enable_dominated != 0 && s->enable_dominated != 1) return fail(h, "invalid settings");
    if (s->enable_parallel_cols != 0 && s->enable_parallel_cols != 1)
        return fail(h, "invalid parallel-column switch");
    if (lp->m < 0 || lp->n < 0 || lp->nnz < 0) return fail(h, "negative size");
    int32_t m = lp->m, n = lp->n;
    if (m > 0 && (!lp->row_ptr || !lp->lhs || !lp->rhs)) return fail(h, "null row array");
    if (n > 0 && (!lp->lb || !lp->ub || !lp->c)) return fail(h, "null column array");
    if (lp->nnz > 0 && (!lp->col_idx || !lp->val)) return fail(h, "null matrix array");
    if (m > 0 && (lp->row_ptr[0] != 0 || lp->row_ptr[m] != lp->nnz)) return fail(h, "bad row_ptr ends");
    if (m == 0 && lp->nnz != 0) return fail(h, "entries without rows");
    for (int32_t i = 0; i < m; ++i) {
        if (lp->row_ptr[i + 1] < lp->row_ptr[i]) return fail(h, "row_ptr decreasing");
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
            int32_t j = lp->col_idx[k];
            if (j < 0 || j >= n) return fail(h, "column index out of range");
            if (k > lp->row_ptr[i] && j <= lp->col_idx[k - 1]) return fail(h, "columns not strictly ascending");
            double a = lp->val[k];
            if (!isfinite(a) || a == 0.0) return fail(h, "coefficient zero or not finite");
        }
    }
    for (int32_t i = 0; i < m; ++i) {
        if (isnan(lp->lhs[i]) || isnan(lp->rhs[i])) return fail(h, "NaN side");
        if (lp->lhs[i] == INFINITY || lp->rhs[i] == -INFINITY) return fail(h, "side infinite on the wrong end");
        if (lp->lhs[i] >= s->inf_value || lp->rhs[i] <= -s->inf_value) return fail(h, "side infinite on the wrong end");
    }
    for (int32_t j = 0; j < n; ++j) {
        if (isnan(lp->lb[j]) || isnan(lp->ub[j])) return fail(h, "NaN bound");
        if (lp->lb[j] >= s->inf_value || lp->ub[j] <= -s->inf_value) return fail(h, "bound infinite on the wrong end");
        if (!isfinite(lp->c[j])) return fail(h, "cost not finite");
    }
    if (!isfinite(lp->obj_offset)) return fail(h, "offset not finite");

    h->m = m; h->n = n; h->nnz = lp->nnz; h->s = *s;
    h->rp = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    h->ci = (int32_t *)xcalloc((size_t)lp->nnz, sizeof(int32_t));
    h->va = (double *)xcalloc((size_t)lp->nnz, sizeof(double));
    h->lhs = (double *)xcalloc((size_t)m, sizeof(double));
    h->rhs = (double *)xcalloc((size_t)m, sizeof(double));
    h->lb = (double *)xcalloc((size_t)n, sizeof(double));
    h->ub = (double *)xcalloc((size_t)n, sizeof(double));
    h->c = (double *)xcalloc((size_t)n, sizeof(double));
    h->c0 = (double *)xcalloc((size_t)n + 1, sizeof(double));
    if (m > 0) memcpy(h->rp, lp->row_ptr, ((size_t)m + 1) * sizeof(int32_t));
    h->ci0 = (int32_t *)xcalloc((size_t)lp->nnz + 1, sizeof(int32_t));
    h->va0 = (double *)xcalloc((size_t)lp->nnz + 1, sizeof(double));
    h->col_mod = (uint8_t *)xcalloc((size_t)n + 1, 1);
    if (lp->nnz > 0) {
        memcpy(h->ci, lp->col_idx, (size_t)lp->nnz * sizeof(int32_t));
        memcpy(h->va, lp->val, (size_t)lp->nnz * sizeof(double));
        memcpy(h->ci0, lp->col_idx, (size_t)lp->nnz * sizeof(int32_t));
        memcpy(h->va0, lp->val, (size_t)lp->nnz * sizeof(double));
    }
    for (int32_t i = 0; i < m; ++i) {
        h->lhs[i] = canon_inf(lp->lhs[i], s->inf_value);
        h->rhs[i] = canon_inf(lp->rhs[i], s->inf_value);
    }
    for (int32_t j = 0; j < n; ++j) {
        h->lb[j] = canon_inf(lp->lb[j], s->inf_value);
        h->ub[j] = canon_inf(lp->ub[j], s->inf_value);
        h->c[j] = pos0(lp->c[j]);
        h->c0[j] = h->c[j];
    }
    h->off = pos0(lp->obj_offset);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* activities (section 3.1): min/max activity with infinite-bound counts      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t L;            /* active (not removed) columns in the row      */
    int32_t ninf_min, ninf_max;
    double minact, maxact; /* pairwise sums of the finite contributions */
} row_stats;

/* contribution of coefficient a on [lo, up] to the min (which=0) / max (1)
 * activity; returns 1 when the bound used is infinite */
static int contribution(double a, double lo, double up, int which, double *out) {
    double b = (a > 0) == (which == 0) ? lo : up;
    if (isinf(b)) { *out = 0.0; return 1; }
    *out = pos0(a * b);
    return 0;
}

static void compute_stats(const or_handle *h, int32_t i, const double *lb, const double *ub,
                          double *tmin, double *tmax, row_stats *st) {
    int64_t s0 = h->rp[i], len = h->rp[i + 1] - h->rp[i];
    st->L = 0; st->ninf_min = 0; st->ninf_max = 0;
    for (int64_t t = 0; t < len; ++t) {
        int32_t j = h->ci[s0 + t];
        double a = h->va[s0 + t];
        if (h->col_on[j]) st->L++;
        st->ninf_min += contribution(a, lb[j], ub[j], 0, &tmin[t]);
        st->ninf_max += contribution(a, lb[j], ub[j], 1, &tmax[t]);
    }
    st->minact = or_pairwise_sum(tmin, len);
    st->maxact = or_pairwise_sum(tmax, len);
}

/* ------------------------------------------------------------------------- */
/* one propagation round (reading R-Jacobi)                                   */
/* ------------------------------------------------------------------------- */

enum { DEC_KEEP = 0, DEC_EMPTY = 1, DEC_REDUNDANT = 2, DEC_SINGLETON = 3, DEC_FORCE_MIN = 4, DEC_FORCE_MAX = 5 };

typedef struct {
    double *lb_s, *ub_s;       /* snapshot                         */
    double *lb_n, *ub_n;       /* best qualifying candidates       */
    int32_t *src_lb, *src_ub;  /* lowest row giving the final value */
    double *tmin, *tmax;       /* per-row scratch                  */
    uint8_t *dec;
    row_stats *st;
    int32_t *down, *up;        /* variable locks (dual fixing)      */
    int32_t *pick;             /* free singleton column of each row */
    int32_t *owner;            /* lowest substituting row of each column */
} round_ws;

/* Implied bounds of row i on each of its active columns, from the residual
 * activity with the column's own contribution taken out. Returns 1 when the
 * row (with one active column) is fully captured by the candidates it gave. */
/* Forcing rows (a primal explorer; Andersen & Andersen 1995, cited by the
 * paper for its explorers): a row with at least two active columns whose
 * finite min activity reaches its rhs (within tol, no infinite contribution)
 * can hold only with every active column at the bound giving its min
 * contribution (a > 0: lb, a < 0: ub); symmetrically a max activity reaching
 * the lhs. Returns 1 (min side) or 2 (max side), else 0. Every active
 * coefficient must be at least coef_tol in magnitude (a tiny one would let
 * its column move far within the tolerance). */
static int forcing_side(const or_handle *h, int32_t i, const row_stats *st) {
    const or_settings *s = &h->s;
    if (!s->enable_forcing_rows || st->L < 2) return 0;
    double lhs = h->lhs[i], rhs = h->rhs[i];
    int side = 0;
    if (st->ninf_min == 0 && !isinf(rhs) && st->minact >= rhs - tol_of(s, rhs)) side = 1;
    else if (st->ninf_max == 0 && !isinf(lhs) && st->maxact <= lhs + tol_of(s, lhs)) side = 2;
    if (!side) return 0;
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
        if (h->col_on[h->ci[k]] && fabs(h->va[k]) < s->coef_tol) return 0;
    return side;
}

/* The forced bounds of a forcing row as candidates: each active column's
 * other bound moves onto the bound its side forces (qualifying whenever it
 * is tighter; the columns are then fixed by the column decisions). */
static void force_row(or_handle *h, int32_t i, int side, round_ws *w) {
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k) {
        int32_t j = h->ci[k];
        if (!h->col_on[j]) continue;
        double a = h->va[k];
        /* min side: a > 0 sits at lb (its ub moves down to lb), a < 0 at ub;
         * max side the other way round */
        int at_lb = (side == 1) == (a > 0);
        if (at_lb) {
            double t_ = w->lb_s[j];
            if (t_ < w->ub_s[j] && t_ < w->ub_n[j]) { w->ub_n[j] = t_; w->src_ub[j] = i; }
        } else {
            double t_ = w->ub_s[j];
            if (t_ > w->lb_s[j] && t_ > w->lb_n[j]) { w->lb_n[j] = t_; w->src_lb[j] = i; }
        }
    }
}

static int propagate_row(or_handle *h, int32_t i, const row_stats *st, round_ws *w) {
    const or_settings *s = &h->s;
    int64_t s0 = h->rp[i], len = h->rp[i + 1] - h->rp[i];
    double lhs = h->lhs[i], rhs = h->rhs[i];
    int single = st->L == 1;
    int captured = 1;
    for (int64_t t = 0; t < len; ++t) {
        int32_t j = h->ci[s0 + t];
        if (!h->col_on[j]) continue;
        double a = h->va[s0 + t];
        if (fabs(a) < s->coef_tol) { captured = 0; continue; }
        double cmin, cmax;
        int imin = contribution(a, w->lb_s[j], w->ub_s[j], 0, &cmin);
        int imax = contribution(a, w->lb_s[j], w->ub_s[j], 1, &cmax);

        /* residual min activity: every other column at its min contribution */
        int have_rmin = 0, have_rmax = 0;
        double rmin = 0, rmax = 0;
        if (st->ninf_min == 0) { rmin = st->minact - cmin; have_rmin = 1; }
        else if (st->ninf_min == 1 && imin) { rmin = st->minact; have_rmin = 1; }
        if (st->ninf_max == 0) { rmax = st->maxact - cmax; have_rmax = 1; }
        else if (st->ninf_max == 1 && imax) { rmax = st->maxact; have_rmax = 1; }

        for (int side = 0; side < 2; ++side) {
            /* side 0: from rhs and the residual min; side 1: from lhs and the residual max */
            double b = side == 0 ? rhs : lhs;
            int have = side == 0 ? have_rmin : have_rmax;
            if (isinf(b)) continue;
            if (!have) { captured = 0; continue; }
            double t_ = pos0((b - (side == 0 ? rmin : rmax)) / a);
            if (!(fabs(t_) < s->inf_value)) { captured = 0; continue; }
            /* a > 0: rhs gives an upper bound, lhs a lower bound; a < 0 swaps */
            int upper = (side == 0) == (a > 0);
            if (upper) {
                double u = w->ub_s[j];
                int q = isinf(u) ? 1 : (single ? t_ < u : t_ < u - s->min_improve * mx1(u));
                if (q && t_ < w->ub_n[j]) { w->ub_n[j] = t_; w->src_ub[j] = i; }
            } else {
                double l = w->lb_s[j];
                int q = isinf(l) ? 1 : (single ? t_ > l : t_ > l + s->min_improve * mx1(l));
                if (q && t_ > w->lb_n[j]) { w->lb_n[j] = t_; w->src_lb[j] = i; }
            }
        }
    }
    return single && captured;
}

static double coef_in_row(const or_handle *h, int32_t i, int32_t j) {
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
        if (h->ci[k] == j) return h->va[k];
    return 0.0;
}

/* Variable locks (section 3.2, "Internal data structures"): down[j] counts
 * the active rows that keep x_j from decreasing -- a > 0 with a finite lhs,
 * or a < 0 with a finite rhs -- and up[j] those that keep it from increasing
 * (a > 0 with a finite rhs, a < 0 with a finite lhs). Recounted from the rows
 * whenever they are needed. */
static void count_locks(const or_handle *h, int32_t *down, int32_t *up) {
    for (int32_t j = 0; j < h->n; ++j) down[j] = up[j] = 0;
    for (int32_t i = 0; i < h->m; ++i) {
        if (!h->row_on[i]) continue;
        int lfin = !isinf(h->lhs[i]), rfin = !isinf(h->rhs[i]);
        for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k) {
            int32_t j = h->ci[k];
            if (h->va[k] > 0) { down[j] += lfin; up[j] += rfin; }
            else { down[j] += rfin; up[j] += lfin; }
        }
    }
}

/* Dual fixing, the lock-based dual reduction (a dominated column): if no
 * active row keeps x_j from moving towards the bound its cost prefers
 * (c_j > 0: down, c_j < 0: up), some optimal solution has x_j at that bound
 * (an infinite one means the LP is unbounded if it is feasible). With
 * c_j = 0 either direction without locks and a finite bound will do, the
 * lower bound first. Returns 1 with the value (possibly infinite) and side. */
static int dual_fix(double c, double lo, double up, int32_t down, int32_t upl, double *v, int *side) {
    if (c > 0 && down == 0) { *v = lo; *side = 0; return 1; }
    if (c < 0 && upl == 0) { *v = up; *side = 1; return 1; }
    if (c == 0 && down == 0 && !isinf(lo)) { *v = lo; *side = 0; return 1; }
    if (c == 0 && upl == 0 && !isinf(up)) { *v = up; *side = 1; return 1; }
    return 0;
}

static void drop_row(or_handle *h, int32_t i) {
    h->row_on[i] = 0;
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
        if (h->col_on[h->ci[k]]) h->col_len[h->ci[k]]--;
}

/* returns 1 if anything changed; sets h->result on infeasible / unbounded */
static int run_round(or_handle *h, round_ws *w) {
    const or_settings *s = &h->s;
    int32_t m = h->m, n = h->n;
    int64_t nrec0 = h->nrec;
    int infeasible = 0, unbounded = 0;

    for (int32_t j = 0; j < n; ++j) {
        w->lb_s[j] = w->lb_n[j] = h->lb[j];
        w->ub_s[j] = w->ub_n[j] = h->ub[j];
        w->src_lb[j] = w->src_ub[j] = -1;
    }

    /* rows: statistics, decisions, propagation (all from the snapshot) */
    for (int32_t i = 0; i < m; ++i) {
        w->dec[i] = DEC_KEEP;
        if (!h->row_on[i]) continue;
        row_stats *st = &w->st[i];
        compute_stats(h, i, w->lb_s, w->ub_s, w->tmin, w->tmax, st);
        double lhs = h->lhs[i], rhs = h->rhs[i];
        int lo_ok = isinf(lhs) || (st->ninf_min == 0 && st->minact >= lhs - tol_of(s, lhs));
        int up_ok = isinf(rhs) || (st->ninf_max == 0 && st->maxact <= rhs + tol_of(s, rhs));
        if (st->L == 0) {
            /* all columns removed: the activity is a constant */
            if (lo_ok && up_ok) w->dec[i] = DEC_EMPTY;
            else infeasible = 1;
            continue;
        }
        if (lo_ok && up_ok) { w->dec[i] = DEC_REDUNDANT; continue; }
        if ((st->ninf_min == 0 && !isinf(rhs) && st->minact > rhs + tol_of(s, rhs)) ||
            (st->ninf_max == 0 && !isinf(lhs) && st->maxact < lhs - tol_of(s, lhs))) {
            infeasible = 1;
            propagate_row(h, i, st, w);
            continue;
        }
        int fs = forcing_side(h, i, st);
        if (fs) {
            w->dec[i] = fs == 1 ? DEC_FORCE_MIN : DEC_FORCE_MAX;
            force_row(h, i, fs, w);
            continue;
        }
        if (propagate_row(h, i, st, w)) w->dec[i] = DEC_SINGLETON;
    }

    /* row records, ascending row index */
    for (int32_t i = 0; i < m; ++i) {
        if (w->dec[i] == DEC_KEEP) continue;
        const row_stats *st = &w->st[i];
        if (w->dec[i] == DEC_EMPTY) {
            push(h, REC_EMPTY_ROW, 0, i, -1, -1, st->minact, h->lhs[i], h->rhs[i], 0);
        } else if (w->dec[i] == DEC_REDUNDANT) {
            push(h, REC_REDUNDANT_ROW, 0, i, -1, -1,
                 st->ninf_min ? -INFINITY : st->minact, st->ninf_max ? INFINITY : st->maxact,
                 h->lhs[i], h->rhs[i]);
        } else if (w->dec[i] == DEC_FORCE_MIN || w->dec[i] == DEC_FORCE_MAX) {
            int mx = w->dec[i] == DEC_FORCE_MAX;
            push(h, REC_FORCING_ROW, mx, i, -1, -1, mx ? st->maxact : st->minact, h->lhs[i], h->rhs[i], 0);
        } else {
            int32_t jj = -1;
            double a = 0;
            for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
                if (h->col_on[h->ci[k]]) { jj = h->ci[k]; a = h->va[k]; }
            push(h, REC_SINGLETON_ROW, 0, i, jj, -1, a, h->lhs[i], h->rhs[i], 0);
        }
        drop_row(h, i);
    }

    /* locks of the rows still active after this round's removals */
    if (s->enable_dual_fix) count_locks(h, w->down, w->up);

    /* columns: bound changes, fixings, empty columns, dual fixings;
     * ascending column index */
    double dv;
    int dside;
    for (int32_t j = 0; j < n; ++j) {
        if (!h->col_on[j]) continue;
        double lo = w->lb_n[j], up = w->ub_n[j];
        if (lo != w->lb_s[j]) {
            push(h, REC_BOUND_CHANGE, 0, -1, j, w->src_lb[j], w->lb_s[j], lo,
                 coef_in_row(h, w->src_lb[j], j), 0);
            h->lsrc[j] = h->lsrc[j] == -1 || h->lsrc[j] == w->src_lb[j] ? w->src_lb[j] : -2;
        }
        if (up != w->ub_s[j]) {
            push(h, REC_BOUND_CHANGE, 1, -1, j, w->src_ub[j], w->ub_s[j], up,
                 coef_in_row(h, w->src_ub[j], j), 0);
            h->usrc[j] = h->usrc[j] == -1 || h->usrc[j] == w->src_ub[j] ? w->src_ub[j] : -2;
        }
        if (!isinf(lo) && !isinf(up) && lo > up + tol_of(s, up)) infeasible = 1;
        if (!isinf(lo) && !isinf(up) && up - lo <= s->fix_tol * mx1(lo)) {
            push(h, REC_FIX_COL, 0, -1, j, -1, lo, h->c[j], 0, 0);
            h->lb[j] = h->ub[j] = lo;
            h->col_on[j] = 0;
        } else if (h->col_len[j] == 0) {
            double cj = h->c[j], v;
            if (cj > 0) v = lo;
            else if (cj < 0) v = up;
            else v = lo > 0 ? lo : (up < 0 ? up : 0.0);
            if (isinf(v)) {
                unbounded = 1;
                h->lb[j] = lo; h->ub[j] = up;
            } else {
                push(h, REC_EMPTY_COL, 0, -1, j, -1, v, cj, 0, 0);
                h->lb[j] = h->ub[j] = v;
                h->col_on[j] = 0;
            }
        } else if (s->enable_dual_fix && dual_fix(h->c[j], lo, up, w->down[j], w->up[j], &dv, &dside)) {
            if (isinf(dv)) {
                unbounded = 1;
                h->lb[j] = lo; h->ub[j] = up;
            } else {
                push(h, REC_DUAL_FIX, dside, -1, j, -1, dv, h->c[j], 0, 0);
                h->lb[j] = h->ub[j] = dv;
                h->col_on[j] = 0;
            }
        } else {
            h->lb[j] = lo;
            h->ub[j] = up;
        }
    }

    /* Free column singletons (section 3.2, "Column singletons"): a column in
     * one alive row i whose bounds are infinite or implied by row i alone
     * (each finite bound came only from tightenings sourced by row i, from an
     * infinite input bound) can absorb any value of row i's other terms
     * within those bounds, so row i and the column leave together; postsolve
     * takes x_j from the row. With c_j != 0 the column is substituted into
     * the objective, x_j = (s - sum_k a_ik x_k) / a_ij with the row's
     * activity s at the side the cost prefers (r = c_j / a_ij > 0: lhs,
     * < 0: rhs; an infinite one: the LP is unbounded if feasible): every
     * other cost of the row becomes c_k - r a_ik and the offset gains r s
     * (the column is kept at s / a_ij with its cost). Such rows claim their
     * columns and one applies only where it is the lowest claimant of each
     * (an independent set by the lowest-index rule; the others wait for the
     * next round). Candidates are read from the state after this round's
     * decisions (rows removed here create none until the next round); a row
     * keeps its lowest candidate. */
    if (s->enable_free_singletons && !infeasible && !unbounded) {
        for (int32_t i = 0; i < m; ++i) w->pick[i] = -1;
        for (int32_t i = 0; i < m; ++i) {
            if (!h->row_on[i]) continue;
            for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k) {
                int32_t j = h->ci[k];
                if (h->col_on[j] && h->col_len[j] == 1 &&
                    (isinf(h->lb[j]) || h->lsrc[j] == i) && (isinf(h->ub[j]) || h->usrc[j] == i)) {
                    w->pick[i] = j;  /* columns ascend within a row: the lowest */
                    break;
                }
            }
        }
        for (int32_t i = 0; i < m; ++i) {
            int32_t j = w->pick[i];
            if (j < 0 || h->c[j] == 0) continue;
            double r = h->c[j] / coef_in_row(h, i, j);
            if (isinf(r > 0 ? h->lhs[i] : h->rhs[i])) unbounded = 1;
        }
        if (!unbounded) {
            for (int32_t j = 0; j < n; ++j) w->owner[j] = INT32_MAX;
            for (int32_t i = 0; i < m; ++i) {
                int32_t j = w->pick[i];
                if (j < 0 || h->c[j] == 0) continue;
                for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
                    if (w->owner[h->ci[k]] > i) w->owner[h->ci[k]] = i;
            }
            for (int32_t i = 0; i < m; ++i) {
                int32_t j = w->pick[i];
                if (j < 0) continue;
                double a = coef_in_row(h, i, j), cj = h->c[j], v = 0.0;
                int side = 0;
                if (cj != 0) {
                    int mine = 1;
                    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k) mine &= w->owner[h->ci[k]] == i;
                    if (!mine) continue;
                    double r = cj / a;
                    side = r > 0 ? 1 : 2;
                    double sv = side == 1 ? h->lhs[i] : h->rhs[i];
                    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
                        if (h->ci[k] != j) h->c[h->ci[k]] = pos0(h->c[h->ci[k]] - r * h->va[k]);
                    v = pos0(sv / a);
                }
                push(h, REC_FREE_SINGLETON, side, i, j, -1, a, h->lhs[i], h->rhs[i], cj);
                h->col_on[j] = 0;
                h->lb[j] = h->ub[j] = v;
                drop_row(h, i);
            }
        }
    }

    if (infeasible) h->result = RES_INFEASIBLE;
    else if (unbounded) h->result = RES_UNBOUNDED;
    return h->nrec != nrec0;
}

/* ------------------------------------------------------------------------- */
/* parallel rows (section 3.2)                                                */
/* ------------------------------------------------------------------------- */

typedef struct { uint64_t key; int32_t row; } keyrow;

static int cmp_keyrow(const void *a, const void *b) {
    const keyrow *x = (const keyrow *)a, *y = (const keyrow *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->row > y->row) - (x->row < y->row);
}

/* Constant contribution of the removed (fixed) columns of row i: the
 * canonical pairwise sum over the row's CSR positions, a removed column's
 * position holding a_ij * v_j and an active one +0. The rows of the current
 * problem are sum over active j of a_ij x_j in [lhs_i - k_i, rhs_i - k_i]
 * (section 3.2, "Internal data structures": inactive columns are ignored
 * when streaming A). Compaction shifts the sides by the same constant. */
static double removed_constant(const or_handle *h, int32_t i, double *tmp) {
    int64_t s0 = h->rp[i], len = h->rp[i + 1] - h->rp[i];
    for (int64_t t = 0; t < len; ++t) {
        int32_t j = h->ci[s0 + t];
        tmp[t] = h->col_on[j] ? 0.0 : pos0(h->va[s0 + t] * h->lb[j]);
    }
    return or_pairwise_sum(tmp, len);
}

/* a side moved by -k (infinite sides stay) */
static double side_minus(double side, double k) { return isinf(side) ? side : pos0(side - k); }
static double side_plus(double side, double k) { return isinf(side) ? side : pos0(side + k); }

/* row i's active entries in CSR order; returns their number */
static int32_t active_entries(const or_handle *h, int32_t i, int32_t *cols, double *vals) {
    int32_t L = 0;
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
        if (h->col_on[h->ci[k]]) {
            cols[L] = h->ci[k];
            vals[L] = h->va[k];
            L++;
        }
    return L;
}

/* Rows r and l of the current problem are parallel when their active entries
 * have the same columns and, each divided by the row's first active
 * coefficient, agree within par_tol (relative to the larger magnitude). */
static int rows_parallel(const or_handle *h, int32_t r, int32_t l, int32_t *cr, double *vr,
                         int32_t *cl, double *vl) {
    int32_t lr = active_entries(h, r, cr, vr), ll = active_entries(h, l, cl, vl);
    if (lr != ll || lr == 0) return 0;
    for (int32_t t = 0; t < lr; ++t) {
        if (cr[t] != cl[t]) return 0;
        double a = vr[t] / vr[0], b = vl[t] / vl[0];
        double scale = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
        if (!(fabs(a - b) <= h->s.par_tol * scale)) return 0;
    }
    return 1;
}

/* first active coefficient of row i (the row has one) */
static double first_active(const or_handle *h, int32_t i) {
    for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k)
        if (h->col_on[h->ci[k]]) return h->va[k];
    return 0.0;
}

/* Parallel rows of the current problem (section 3.2, "Parallel rows"):
 * rows with a_r = lambda a_L over their active entries. Key = the two-level
 * hash of the active entries; leader of a key group = its lowest equality
 * row, else its lowest row; every other row of the group is verified
 * against the leader. With k = the removed-column constant of a row, a
 * verified row r maps its effective sides [lhs_r - k_r, rhs_r - k_r] through
 * lambda = (first active a_r) / (first active a_L) (lambda < 0 swaps them);
 * the leader's effective sides become the intersection with its own, the
 * source of each side being the lowest row that gives it. A side the leader
 * keeps keeps its stored value; a side from another row is stored as
 * effective + k_L. Returns 1 if any row was merged. */
static int parallel_rows(or_handle *h) {
    const or_settings *s = &h->s;
    int32_t m = h->m;
    int64_t maxlen = 1;
    for (int32_t i = 0; i < m; ++i)
        if (h->rp[i + 1] - h->rp[i] > maxlen) maxlen = h->rp[i + 1] - h->rp[i];
    int32_t *c1 = (int32_t *)xcalloc((size_t)maxlen, sizeof(int32_t));
    int32_t *c2 = (int32_t *)xcalloc((size_t)maxlen, sizeof(int32_t));
    double *v1 = (double *)xcalloc((size_t)maxlen, sizeof(double));
    double *v2 = (double *)xcalloc((size_t)maxlen, sizeof(double));
    keyrow *kr = (keyrow *)xcalloc((size_t)m + 1, sizeof(keyrow));
    int32_t nk = 0;
    for (int32_t i = 0; i < m; ++i) {
        if (!h->row_on[i]) continue;
        int32_t L = active_entries(h, i, c1, v1);
        if (L < 2) continue;
        kr[nk].key = or_row_key(c1, v1, L);
        kr[nk].row = i;
        nk++;
    }
    qsort(kr, (size_t)nk, sizeof(keyrow), cmp_keyrow);

    int32_t *leader_of = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    double *lam = (double *)xcalloc((size_t)m + 1, sizeof(double));
    double *new_l = (double *)xcalloc((size_t)m + 1, sizeof(double));
    double *new_u = (double *)xcalloc((size_t)m + 1, sizeof(double));
    int32_t *src_l = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    int32_t *src_u = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    double *kconst = (double *)xcalloc((size_t)m + 1, sizeof(double));
    uint8_t *is_leader = (uint8_t *)xcalloc((size_t)m + 1, 1);
    for (int32_t i = 0; i < m; ++i) leader_of[i] = -1;

    for (int32_t g0 = 0; g0 < nk;) {
        int32_t g1 = g0 + 1;
        while (g1 < nk && kr[g1].key == kr[g0].key) g1++;
        if (g1 - g0 >= 2) {
            /* leader: the first equality row of the group, else the first row */
            int32_t L = -1;
            for (int32_t t = g0; t < g1 && L < 0; ++t)
                if (h->lhs[kr[t].row] == h->rhs[kr[t].row]) L = kr[t].row;
            if (L < 0) L = kr[g0].row;
            double kL = removed_constant(h, L, v1);
            /* members in ascending row order; the leader's own sides first */
            double lo = side_minus(h->lhs[L], kL), up = side_minus(h->rhs[L], kL);
            int32_t sl = L, su = L;
            int any = 0;
            for (int32_t t = g0; t < g1; ++t) {
                int32_t r = kr[t].row;
                if (r == L || !rows_parallel(h, r, L, c1, v1, c2, v2)) continue;
                double kr_ = removed_constant(h, r, v1);
                double el = side_minus(h->lhs[r], kr_), eu = side_minus(h->rhs[r], kr_);
                double la = first_active(h, r) / first_active(h, L);
                double ml, mu;
                if (la > 0) { ml = el / la; mu = eu / la; }
                else { ml = eu / la; mu = el / la; }
                ml = pos0(ml); mu = pos0(mu);
                if (ml > lo || (ml == lo && r < sl)) { lo = ml; sl = r; }
                if (mu < up || (mu == up && r < su)) { up = mu; su = r; }
                leader_of[r] = L;
                lam[r] = la;
                any = 1;
            }
            if (any) {
                is_leader[L] = 1;
                new_l[L] = lo; new_u[L] = up;
                src_l[L] = sl; src_u[L] = su;
                kconst[L] = kL;
            }
        }
        g0 = g1;
    }

    int merged = 0, infeasible = 0;
    for (int32_t i = 0; i < m; ++i) {
        if (leader_of[i] >= 0) {
            push(h, REC_PARALLEL_ROW, 0, i, -1, leader_of[i], lam[i], h->lhs[i], h->rhs[i], 0);
            drop_row(h, i);
            merged = 1;
        } else if (is_leader[i]) {
            double lo = new_l[i], up = new_u[i];
            int snapped = 0;
            if (!isinf(lo) && !isinf(up) && lo > up) {
                if (lo > up + tol_of(s, up)) infeasible = 1;
                else { lo = up; snapped = 1; }
            }
            /* back to stored sides: a side the leader gave itself is kept */
            double nu = src_u[i] == i ? h->rhs[i] : side_plus(up, kconst[i]);
            double nl = snapped ? nu : (src_l[i] == i ? h->lhs[i] : side_plus(lo, kconst[i]));
            if (nl != h->lhs[i] || nu != h->rhs[i]) {
                push(h, REC_LEADER_SIDES, 0, i, src_l[i], src_u[i], h->lhs[i], h->rhs[i], nl, nu);
                h->lhs[i] = nl;
                h->rhs[i] = nu;
            }
        }
    }
    if (infeasible) h->result = RES_INFEASIBLE;
    free(kr); free(leader_of); free(lam); free(new_l); free(new_u);
    free(src_l); free(src_u); free(is_leader); free(kconst);
    free(c1); free(c2); free(v1); free(v2);
    return merged;
}

/* ------------------------------------------------------------------------- */
/* parallel columns (section 3.2): parallel rows of [c A'] -- columns j, k   */
/* with a_j = lambda a_k and c_j = lambda c_k -- merge into one variable     */
/* x_k + lambda x_j whose bounds are the sum of the intervals.               */
/* ------------------------------------------------------------------------- */

/* first entry of column j's augmented row [c_j, a_ij over alive rows i] */
static double col_first(const or_handle *h, int32_t j) {
    if (h->c[j] != 0) return h->c[j];
    for (int32_t q = h->cp[j]; q < h->cp[j + 1]; ++q)
        if (h->row_on[h->ri[q]]) return h->cva[q];
    return 0.0;
}

/* 63-bit key of the augmented row: the parallel-row key over its entries,
 * with the cost as an entry of id 2^32 - 1 before the rows, normalised by the
 * first entry, top 63 bits (columns that are not candidates sort after every
 * key) */
static uint64_t col_key(const or_handle *h, int32_t j) {
    double f = col_first(h, j);
    uint64_t h1 = 0, h2 = 0;
    if (h->c[j] != 0) {
        uint64_t id = splitmix(0xFFFFFFFFULL);
        h1 += 1 + id;
        h2 += splitmix(id ^ quantize(h->c[j] / f));
    }
    for (int32_t q = h->cp[j]; q < h->cp[j + 1]; ++q) {
        if (!h->row_on[h->ri[q]]) continue;
        uint64_t id = splitmix((uint64_t)(uint32_t)h->ri[q]);
        h1 += 1 + id;
        h2 += splitmix(id ^ quantize(h->cva[q] / f));
    }
    return (splitmix(h1) ^ h2) >> 1;
}

/* same augmented pattern and entries within par_tol after normalisation */
static int cols_parallel(const or_handle *h, int32_t j, int32_t k) {
    if ((h->c[j] != 0) != (h->c[k] != 0)) return 0;
    double fj = col_first(h, j), fk = col_first(h, k);
    int32_t qj = h->cp[j], qk = h->cp[k];
    for (;;) {
        while (qj < h->cp[j + 1] && !h->row_on[h->ri[qj]]) qj++;
        while (qk < h->cp[k + 1] && !h->row_on[h->ri[qk]]) qk++;
        int ej = qj < h->cp[j + 1], ek = qk < h->cp[k + 1];
        if (ej != ek) return 0;
        if (!ej) break;
        if (h->ri[qj] != h->ri[qk]) return 0;
        double a = h->cva[qj] / fj, b = h->cva[qk] / fk;
        double scale = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
        if (!(fabs(a - b) <= h->s.par_tol * scale)) return 0;
        qj++;
        qk++;
    }
    return 1;
}

/* a merged bound: |v| >= inf_value is infinite, -0 is +0 */
static double canon_bound(const or_handle *h, double v) {
    if (fabs(v) >= h->s.inf_value) return v > 0 ? INFINITY : -INFINITY;
    return pos0(v);
}

/* interval of the merged variable after adding lambda * [lb, ub] */
static void add_scaled(const or_handle *h, double lam, double lb, double ub, double *lo, double *up) {
    if (lam > 0) {
        *lo = canon_bound(h, *lo + lam * lb);
        *up = canon_bound(h, *up + lam * ub);
    } else {
        *lo = canon_bound(h, *lo + lam * ub);
        *up = canon_bound(h, *up + lam * lb);
    }
}

typedef struct { uint64_t key; int32_t col; } keycol;

static int cmp_keycol(const void *a, const void *b) {
    const keycol *x = (const keycol *)a, *y = (const keycol *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->col > y->col) - (x->col < y->col);
}

/* Candidates: active columns in at least one alive row, of any length (the
 * paper sets no limit). Groups: equal keys, in ascending column order; the
 * leader is the group's first column, every other member is verified
 * against it and merged into it in ascending order. Records in one pass
 * over the columns: LEADER_BOUNDS for a leader, PARALLEL_COL for a merged
 * column. Returns 1 if any column merged. */
static int parallel_cols(or_handle *h) {
    int32_t n = h->n;
    keycol *kc = (keycol *)xcalloc((size_t)n + 1, sizeof(keycol));
    int32_t nk = 0;
    for (int32_t j = 0; j < n; ++j) {
        if (!h->col_on[j] || h->col_len[j] < 1) continue;
        kc[nk].key = col_key(h, j);
        kc[nk].col = j;
        nk++;
    }
    qsort(kc, (size_t)nk, sizeof(keycol), cmp_keycol);
    int32_t *lead = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    double *lam = (double *)xcalloc((size_t)n + 1, sizeof(double));
    double *nlo = (double *)xcalloc((size_t)n + 1, sizeof(double));
    double *nup = (double *)xcalloc((size_t)n + 1, sizeof(double));
    for (int32_t j = 0; j < n; ++j) lead[j] = -1;
    for (int32_t g0 = 0; g0 < nk;) {
        int32_t g1 = g0 + 1;
        while (g1 < nk && kc[g1].key == kc[g0].key) g1++;
        int32_t k = kc[g0].col;
        double lo = h->lb[k], up = h->ub[k];
        double fk = col_first(h, k);
        int any = 0;
        for (int32_t t = g0 + 1; t < g1; ++t) {
            int32_t j = kc[t].col;
            if (!cols_parallel(h, j, k)) continue;
            double la = col_first(h, j) / fk;
            add_scaled(h, la, h->lb[j], h->ub[j], &lo, &up);
            lead[j] = k;
            lam[j] = la;
            any = 1;
        }
        if (any && (!(lo < INFINITY) || !(up > -INFINITY))) {
            /* the merged interval passed inf_value on the wrong side: no
             * finite value would satisfy it, so the group is not merged. A
             * lower sum that reached +inf and then met a -inf term is NaN
             * (and the mirror for the upper sum): not merged either. */
            for (int32_t t = g0 + 1; t < g1; ++t)
                if (lead[kc[t].col] == k) lead[kc[t].col] = -1;
            any = 0;
        }
        if (any) {
            lead[k] = k;
            nlo[k] = lo;
            nup[k] = up;
        }
        g0 = g1;
    }
    int merged = 0;
    for (int32_t j = 0; j < n; ++j) {
        if (lead[j] < 0) continue;
        if (lead[j] == j) {
            push(h, REC_LEADER_BOUNDS, 0, -1, j, -1, h->lb[j], h->ub[j], nlo[j], nup[j]);
            h->lb[j] = nlo[j];
            h->ub[j] = nup[j];
            h->lsrc[j] = isinf(nlo[j]) ? -1 : -2;
            h->usrc[j] = isinf(nup[j]) ? -1 : -2;
        } else {
            push(h, REC_PARALLEL_COL, 0, -1, j, lead[j], lam[j], h->lb[j], h->ub[j], 0);
            h->col_on[j] = 0;
            h->lb[j] = h->ub[j] = 0.0;
            merged = 1;
        }
    }
    free(kc); free(lead); free(lam); free(nlo); free(nup);
    return merged;
}

/* ------------------------------------------------------------------------- */
/* dominated columns through implied dual bounds (a dual explorer, section    */
/* 2.1; reading R-DomCol)                                                     */
/* ------------------------------------------------------------------------- */

/* Bounds on the row duals y (c - A'y - z = 0) that every optimal solution of
 * the current problem satisfies: an alive row with only a finite lhs has
 * y_i >= 0, with only a finite rhs y_i <= 0; and an active column j in one
 * alive row i (coefficient a, |a| >= coef_tol) has z_j >= 0 when ub_j = +inf
 * and z_j <= 0 when lb_j = -inf, i.e. a y_i <= c_j, resp. a y_i >= c_j.
 * Then for every active column k in at least one alive row, z_k lies in
 * [c_k - sum_i max(a_ik y_i), c_k - sum_i min(a_ik y_i)] over those bounds
 * (each sum canonical pairwise over the column's stored positions, the other
 * positions contributing +0; an infinite term makes that end infinite). A
 * lower end above feas_tol * max(1, |c_k|) puts x_k at its lower bound in
 * every optimal solution, an upper end below -feas_tol * max(1, |c_k|) at its
 * upper bound; an infinite such bound means the LP is unbounded if feasible.
 * All fixings of the pass are taken from the problem before it (each holds
 * in every optimal solution, so together too); records in column order. The
 * bounds hold for every dual-feasible y, so bounds of a row that cross by
 * more than feas_tol * max(1, |upper|) leave no dual solution: the LP is
 * unbounded if it is feasible; a smaller crossing changes nothing. */
static int dominated_cols(or_handle *h) {
    const or_settings *s = &h->s;
    int32_t m = h->m, n = h->n;
    double *ylo = (double *)xcalloc((size_t)m + 1, sizeof(double));
    double *yhi = (double *)xcalloc((size_t)m + 1, sizeof(double));
    for (int32_t i = 0; i < m; ++i) {
        ylo[i] = yhi[i] = 0.0;
        if (!h->row_on[i]) continue;
        int lf = !isinf(h->lhs[i]), rf = !isinf(h->rhs[i]);
        if (!lf && !rf) continue;
        ylo[i] = lf && !rf ? 0.0 : -INFINITY;
        yhi[i] = rf && !lf ? 0.0 : INFINITY;
    }
    for (int32_t j = 0; j < n; ++j) {
        if (!h->col_on[j] || h->col_len[j] != 1) continue;
        int32_t i = -1;
        double a = 0.0;
        for (int32_t q = h->cp[j]; q < h->cp[j + 1]; ++q)
            if (h->row_on[h->ri[q]]) { i = h->ri[q]; a = h->cva[q]; }
        if (i < 0 || fabs(a) < s->coef_tol) continue;
        double v = h->c[j] / a;
        if (isinf(h->ub[j])) {
            if (a > 0) yhi[i] = v < yhi[i] ? v : yhi[i];
            else ylo[i] = v > ylo[i] ? v : ylo[i];
        }
        if (isinf(h->lb[j])) {
            if (a > 0) ylo[i] = v > ylo[i] ? v : ylo[i];
            else yhi[i] = v < yhi[i] ? v : yhi[i];
        }
    }
    for (int32_t i = 0; i < m; ++i)
        if (ylo[i] > yhi[i]) {
            if (ylo[i] > yhi[i] + tol_of(s, yhi[i])) h->result = RES_UNBOUNDED;
            free(ylo); free(yhi);
            return 0;
        }
    int64_t maxlen = 0;
    for (int32_t j = 0; j < n; ++j)
        if (h->cp[j + 1] - h->cp[j] > maxlen) maxlen = h->cp[j + 1] - h->cp[j];
    double *thi = (double *)xcalloc((size_t)maxlen + 1, sizeof(double));
    double *tlo = (double *)xcalloc((size_t)maxlen + 1, sizeof(double));
    int8_t *side = (int8_t *)xcalloc((size_t)n + 1, 1);
    for (int32_t k = 0; k < n; ++k) {
        side[k] = -1;
        if (!h->col_on[k] || h->col_len[k] < 1) continue;
        int64_t len = h->cp[k + 1] - h->cp[k];
        int inf_hi = 0, inf_lo = 0;
        for (int64_t t = 0; t < len; ++t) {
            int32_t q = h->cp[k] + (int32_t)t;
            double a = h->cva[q];
            int32_t i = h->ri[q];
            thi[t] = tlo[t] = 0.0;
            if (!h->row_on[i] || a == 0.0) continue;
            double hi = a > 0 ? a * yhi[i] : a * ylo[i];  /* max of a y_i */
            double lo = a > 0 ? a * ylo[i] : a * yhi[i];  /* min of a y_i */
            if (isinf(hi)) inf_hi++; else thi[t] = pos0(hi);
            if (isinf(lo)) inf_lo++; else tlo[t] = pos0(lo);
        }
        double ck = h->c[k], tol = tol_of(s, ck);
        if (inf_hi == 0 && ck - or_pairwise_sum(thi, len) > tol) side[k] = 0;
        else if (inf_lo == 0 && ck - or_pairwise_sum(tlo, len) < -tol) side[k] = 1;
    }
    int any = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (side[k] < 0) continue;
        double v = side[k] == 0 ? h->lb[k] : h->ub[k];
        if (isinf(v)) {
            h->result = RES_UNBOUNDED;
            continue;
        }
        push(h, REC_DOMINATED_COL, side[k], -1, k, -1, v, h->c[k], 0, 0);
        h->lb[k] = h->ub[k] = v;
        h->col_on[k] = 0;
        any = 1;
    }
    free(ylo); free(yhi); free(thi); free(tlo); free(side);
    return any;
}

/* ------------------------------------------------------------------------- */
/* reduced problem (section 3.3)                                              */
/* ------------------------------------------------------------------------- */

static void compact(or_handle *h) {
    int32_t m = h->m, n = h->n;
    int32_t *nr = (int32_t *)xcalloc((size_t)m, sizeof(int32_t));
    int32_t *nc = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    int32_t rm = 0, rn = 0;
    for (int32_t i = 0; i < m; ++i) nr[i] = h->row_on[i] ? rm++ : -1;
    for (int32_t j = 0; j < n; ++j) nc[j] = h->col_on[j] ? rn++ : -1;
    int64_t rnnz = 0;
    for (int32_t i = 0; i < m; ++i)
        if (h->row_on[i])
            for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k) rnnz += h->col_on[h->ci[k]];

    h->rm = rm; h->rn = rn; h->rnnz = rnnz;
    h->r_rp = (int32_t *)xcalloc((size_t)rm + 1, sizeof(int32_t));
    h->r_ci = (int32_t *)xcalloc((size_t)rnnz, sizeof(int32_t));
    h->r_va = (double *)xcalloc((size_t)rnnz, sizeof(double));
    h->r_cp = (int32_t *)xcalloc((size_t)rn + 1, sizeof(int32_t));
    h->r_ri = (int32_t *)xcalloc((size_t)rnnz, sizeof(int32_t));
    h->r_cva = (double *)xcalloc((size_t)rnnz, sizeof(double));
    h->r_lhs = (double *)xcalloc((size_t)rm, sizeof(double));
    h->r_rhs = (double *)xcalloc((size_t)rm, sizeof(double));
    h->r_lb = (double *)xcalloc((size_t)rn, sizeof(double));
    h->r_ub = (double *)xcalloc((size_t)rn, sizeof(double));
    h->r_c = (double *)xcalloc((size_t)rn, sizeof(double));
    h->r_rowmap = (int32_t *)xcalloc((size_t)rm, sizeof(int32_t));
    h->r_colmap = (int32_t *)xcalloc((size_t)rn, sizeof(int32_t));
    h->r_rcls = (uint8_t *)xcalloc((size_t)rm, 1);
    h->r_ccls = (uint8_t *)xcalloc((size_t)rn, 1);

    int64_t maxlen = 0;
    for (int32_t i = 0; i < m; ++i)
        if (h->rp[i + 1] - h->rp[i] > maxlen) maxlen = h->rp[i + 1] - h->rp[i];
    double *tmp = (double *)xcalloc((size_t)maxlen, sizeof(double));

    int64_t pos = 0;
    for (int32_t i = 0; i < m; ++i) {
        if (!h->row_on[i]) continue;
        int32_t ri = nr[i];
        h->r_rowmap[ri] = i;
        for (int64_t q = h->rp[i]; q < h->rp[i + 1]; ++q) {
            int32_t j = h->ci[q];
            if (h->col_on[j]) {
                h->r_ci[pos] = nc[j];
                h->r_va[pos] = h->va[q];
                pos++;
            }
        }
        h->r_rp[ri + 1] = (int32_t)pos;
        /* sides shifted by the removed columns' constant contribution */
        double k = removed_constant(h, i, tmp);
        h->r_lhs[ri] = side_minus(h->lhs[i], k);
        h->r_rhs[ri] = side_minus(h->rhs[i], k);
        int32_t L = h->r_rp[ri + 1] - h->r_rp[ri];
        h->r_rcls[ri] = L == 1 ? RCLS_SINGLETON
                      : L == 2 ? (h->r_lhs[ri] == h->r_rhs[ri] ? RCLS_DOUBLETON_EQ : RCLS_DOUBLETON_INEQ)
                      : RCLS_OTHER;
    }
    free(tmp);

    /* objective offset: removed columns' cost terms, pairwise over j */
    double *terms = (double *)xcalloc((size_t)n, sizeof(double));
    for (int32_t j = 0; j < n; ++j) {
        if (h->col_on[j]) {
            terms[j] = 0.0;
            int32_t rj = nc[j];
            h->r_colmap[rj] = j;
            h->r_lb[rj] = h->lb[j];
            h->r_ub[rj] = h->ub[j];
            h->r_c[rj] = h->c[j];
        } else {
            terms[j] = pos0(h->c[j] * h->lb[j]);
        }
    }
    h->roff = pos0(h->off + or_pairwise_sum(terms, n));
    free(terms);

    /* CSC of the reduced matrix: stable counting transpose */
    for (int64_t p = 0; p < rnnz; ++p) h->r_cp[h->r_ci[p] + 1]++;
    for (int32_t j = 0; j < rn; ++j) h->r_cp[j + 1] += h->r_cp[j];
    int32_t *cur = (int32_t *)xcalloc((size_t)rn + 1, sizeof(int32_t));
    memcpy(cur, h->r_cp, ((size_t)rn + 1) * sizeof(int32_t));
    for (int32_t ri = 0; ri < rm; ++ri)
        for (int64_t p = h->r_rp[ri]; p < h->r_rp[ri + 1]; ++p) {
            int32_t cj = h->r_ci[p];
            h->r_ri[cur[cj]] = ri;
            h->r_cva[cur[cj]] = h->r_va[p];
            cur[cj]++;
        }
    free(cur);
    for (int32_t rj = 0; rj < rn; ++rj) {
        int32_t len = h->r_cp[rj + 1] - h->r_cp[rj];
        int free_col = isinf(h->r_lb[rj]) && isinf(h->r_ub[rj]);
        h->r_ccls[rj] = len == 1 ? (free_col ? CCLS_SINGLETON_FREE : CCLS_SINGLETON)
                      : len == 2 ? CCLS_DOUBLETON : CCLS_OTHER;
    }
    free(nr);
    free(nc);
}

/* ------------------------------------------------------------------------- */
/* driver                                                                     */
/* ------------------------------------------------------------------------- */

/* the matrix by columns from the (current) rows: rows ascending within a
 * column */
static void build_columns(or_handle *h) {
    int32_t m = h->m, n = h->n;
    memset(h->cp, 0, ((size_t)n + 1) * sizeof(int32_t));
    for (int64_t k = 0; k < h->nnz; ++k) h->cp[h->ci[k] + 1]++;
    for (int32_t j = 0; j < n; ++j) h->cp[j + 1] += h->cp[j];
    int32_t *fill = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int32_t j = 0; j < n; ++j) fill[j] = h->cp[j];
    for (int32_t i = 0; i < m; ++i)
        for (int32_t k = h->rp[i]; k < h->rp[i + 1]; ++k) {
            int32_t q = fill[h->ci[k]]++;
            h->ri[q] = i;
            h->cva[q] = h->va[k];
        }
    free(fill);
}

/* ------------------------------------------------------------------------- */
/* doubleton equalities (section 2.1, "Explorers": the doubleton-row explorer */
/* uses an equality with two nonzeros to eliminate one of its variables)      */
/* ------------------------------------------------------------------------- */

/* position of column j in row i (ascending columns), or -1 */
static int64_t find_in_row(const or_handle *h, int32_t i, int32_t j) {
    int64_t lo = h->rp[i], hi = h->rp[i + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (h->ci[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return lo < h->rp[i + 1] && h->ci[lo] == j ? lo : -1;
}

/* Row r loses column k and gains coefficient v on column j, in place: with j
 * already in the row its coefficient becomes v and k's entry turns into a
 * dead entry (column k, coefficient +0: k is removed, so the entry adds +0
 * to every sum); otherwise k's entry is taken out and j inserted at its
 * sorted place, the entries between moving by one. The row keeps its
 * length. Returns 1 when j was inserted. */
static int rewrite_row(or_handle *h, int32_t r, int32_t k, int32_t j, double v) {
    int64_t pk = find_in_row(h, r, k), pj = find_in_row(h, r, j);
    if (pj >= 0) {
        h->va[pj] = v;
        h->va[pk] = 0.0;
        return 0;
    }
    if (j > k) {
        int64_t q = pk;
        while (q + 1 < h->rp[r + 1] && h->ci[q + 1] < j) {
            h->ci[q] = h->ci[q + 1];
            h->va[q] = h->va[q + 1];
            q++;
        }
        h->ci[q] = j;
        h->va[q] = v;
    } else {
        int64_t q = pk;
        while (q > h->rp[r] && h->ci[q - 1] > j) {
            h->ci[q] = h->ci[q - 1];
            h->va[q] = h->va[q - 1];
            q--;
        }
        h->ci[q] = j;
        h->va[q] = v;
    }
    return 1;
}

/* The substitution pass (after the parallel passes of an outer cycle).
 * Candidates: alive rows with lhs = rhs (finite) and exactly two active
 * columns, both |a| >= coef_tol, neither a column kept by an earlier
 * substitution (its entries were rewritten). The row is a_j x_j + a_k x_k = b
 * with b = rhs - (the removed columns' constant). Eliminated: the column in
 * fewer alive rows, then the one with the larger |a|, then the lower index;
 * the other is kept. A candidate is dropped when rewriting one of its rows
 * would cancel a coefficient to exactly zero. Conflicts: each candidate
 * claims its two columns and every alive row of the eliminated column; it
 * applies when it is the lowest-index claimant of all of them (the others
 * wait for a later cycle). Applying (x_k = (b - a_j x_j) / a_k):
 *   - each other alive row r of column k, with f = a_rk / a_k, gets
 *     a_rj - f a_j on column j (inserted when absent) and loses k, its sides
 *     moving by f b;
 *   - x_k's bounds move to x_j: (b - a_k bound) / a_j for each finite bound
 *     of k becomes a bound of j when strictly tighter (BOUND_CHANGE from row
 *     i); a value with |v| >= inf_value gives none;
 *   - costs: with r = c_k / a_k, c_j becomes c_j - r a_j; column k leaves at
 *     the value b / a_k (its cost stays, so the offset gains c_k b / a_k);
 *   - row i leaves.
 * Records: DOUBLETON_ROW in ascending row order, then the transferred bounds
 * in ascending column order (lower, then upper). Returns 1 when any
 * substitution applied. */
static int doubleton_pass(or_handle *h) {
    const or_settings *s = &h->s;
    int32_t m = h->m, n = h->n;
    int64_t maxlen = 1;
    for (int32_t i = 0; i < m; ++i)
        if (h->rp[i + 1] - h->rp[i] > maxlen) maxlen = h->rp[i + 1] - h->rp[i];
    int32_t *cols = (int32_t *)xcalloc((size_t)maxlen, sizeof(int32_t));
    double *vals = (double *)xcalloc((size_t)maxlen, sizeof(double));
    int32_t *cj = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    int32_t *ck = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    double *aj = (double *)xcalloc((size_t)m + 1, sizeof(double));
    double *ak = (double *)xcalloc((size_t)m + 1, sizeof(double));
    double *bb = (double *)xcalloc((size_t)m + 1, sizeof(double));
    int32_t *row_claim = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    int32_t *col_claim = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int32_t i = 0; i < m; ++i) { cj[i] = -1; row_claim[i] = INT32_MAX; }
    for (int32_t j = 0; j < n; ++j) col_claim[j] = INT32_MAX;

    /* candidates */
    for (int32_t i = 0; i < m; ++i) {
        if (!h->row_on[i] || h->lhs[i] != h->rhs[i] || isinf(h->rhs[i])) continue;
        if (active_entries(h, i, cols, vals) != 2) continue;
        if (fabs(vals[0]) < s->coef_tol || fabs(vals[1]) < s->coef_tol) continue;
        if (h->col_mod[cols[0]] || h->col_mod[cols[1]]) continue;
        int e;  /* index of the eliminated one among the two */
        int32_t l0 = h->col_len[cols[0]], l1 = h->col_len[cols[1]];
        if (l0 != l1) e = l0 < l1 ? 0 : 1;
        else if (fabs(vals[0]) != fabs(vals[1])) e = fabs(vals[0]) > fabs(vals[1]) ? 0 : 1;
        else e = 0;  /* the lower column index */
        int32_t k = cols[e], j = cols[1 - e];
        double a_k = vals[e], a_j = vals[1 - e];
        /* no rewritten coefficient may cancel to zero */
        int cancels = 0;
        for (int32_t q = h->cp[k]; q < h->cp[k + 1] && !cancels; ++q) {
            int32_t r = h->ri[q];
            if (r == i || !h->row_on[r]) continue;
            int64_t pj = find_in_row(h, r, j);
            if (pj >= 0 && h->va[pj] - (h->cva[q] / a_k) * a_j == 0.0) cancels = 1;
        }
        if (cancels) continue;
        cj[i] = j; ck[i] = k; aj[i] = a_j; ak[i] = a_k;
        bb[i] = side_minus(h->rhs[i], removed_constant(h, i, vals));
    }
    /* claims */
    for (int32_t i = 0; i < m; ++i) {
        if (cj[i] < 0) continue;
        if (i < col_claim[cj[i]]) col_claim[cj[i]] = i;
        if (i < col_claim[ck[i]]) col_claim[ck[i]] = i;
        for (int32_t q = h->cp[ck[i]]; q < h->cp[ck[i] + 1]; ++q) {
            int32_t r = h->ri[q];
            if (h->row_on[r] && i < row_claim[r]) row_claim[r] = i;
        }
    }
    int any = 0;
    for (int32_t i = 0; i < m; ++i) {
        if (cj[i] < 0) continue;
        int own = col_claim[cj[i]] == i && col_claim[ck[i]] == i;
        for (int32_t q = h->cp[ck[i]]; q < h->cp[ck[i] + 1] && own; ++q) {
            int32_t r = h->ri[q];
            if (h->row_on[r] && row_claim[r] != i) own = 0;
        }
        if (!own) { cj[i] = -1; continue; }
        any = 1;
        push(h, REC_DOUBLETON_ROW, 0, i, cj[i], ck[i], aj[i], ak[i], bb[i], h->c[ck[i]]);
    }
    if (!any) goto done;

    /* transferred bounds of the kept columns, ascending column order */
    {
        double *tlo = (double *)xcalloc((size_t)n + 1, sizeof(double));
        double *thi = (double *)xcalloc((size_t)n + 1, sizeof(double));
        int32_t *by = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
        for (int32_t j = 0; j < n; ++j) by[j] = -1;
        for (int32_t i = 0; i < m; ++i) {
            if (cj[i] < 0) continue;
            int32_t j = cj[i], k = ck[i];
            double lo = -INFINITY, hi = INFINITY;
            /* x_j = (b - a_k x_k) / a_j is decreasing in x_k when a_k / a_j > 0 */
            int dec = (ak[i] > 0) == (aj[i] > 0);
            double from_lb = isinf(h->lb[k]) ? (dec ? INFINITY : -INFINITY)
                                             : pos0((bb[i] - ak[i] * h->lb[k]) / aj[i]);
            double from_ub = isinf(h->ub[k]) ? (dec ? -INFINITY : INFINITY)
                                             : pos0((bb[i] - ak[i] * h->ub[k]) / aj[i]);
            if (dec) { lo = from_ub; hi = from_lb; }
            else { lo = from_lb; hi = from_ub; }
            if (fabs(lo) >= s->inf_value) lo = -INFINITY;
            if (fabs(hi) >= s->inf_value) hi = INFINITY;
            tlo[j] = lo; thi[j] = hi; by[j] = i;
        }
        for (int32_t j = 0; j < n; ++j) {
            int32_t i = by[j];
            if (i < 0) continue;
            if (tlo[j] > h->lb[j]) {
                push(h, REC_BOUND_CHANGE, 0, -1, j, i, h->lb[j], tlo[j], aj[i], 0);
                h->lb[j] = tlo[j];
                h->lsrc[j] = h->lsrc[j] == -1 || h->lsrc[j] == i ? i : -2;
            }
            if (thi[j] < h->ub[j]) {
                push(h, REC_BOUND_CHANGE, 1, -1, j, i, h->ub[j], thi[j], aj[i], 0);
                h->ub[j] = thi[j];
                h->usrc[j] = h->usrc[j] == -1 || h->usrc[j] == i ? i : -2;
            }
            if (!isinf(h->lb[j]) && !isinf(h->ub[j]) && h->lb[j] > h->ub[j] + tol_of(s, h->ub[j]))
                h->result = RES_INFEASIBLE;
        }
        free(tlo); free(thi); free(by);
    }
    /* rows, costs, the eliminated columns, the equality rows */
    for (int32_t i = 0; i < m; ++i) {
        if (cj[i] < 0) continue;
        int32_t j = cj[i], k = ck[i];
        for (int32_t q = h->cp[k]; q < h->cp[k + 1]; ++q) {
            int32_t r = h->ri[q];
            if (r == i || !h->row_on[r]) continue;
            double f = h->cva[q] / ak[i];
            int64_t pj = find_in_row(h, r, j);
            double v = (pj >= 0 ? h->va[pj] : 0.0) - f * aj[i];
            double sh = f * bb[i];
            h->lhs[r] = side_minus(h->lhs[r], sh);
            h->rhs[r] = side_minus(h->rhs[r], sh);
            h->col_len[j] += rewrite_row(h, r, k, j, v);
        }
        double rc = h->c[k] / ak[i];
        h->c[j] = pos0(h->c[j] - rc * aj[i]);
        h->col_mod[j] = 1;
        drop_row(h, i);
        double vk = pos0(bb[i] / ak[i]);
        h->col_on[k] = 0;
        h->lb[k] = h->ub[k] = vk;
    }
    build_columns(h);
done:
    free(cols); free(vals); free(cj); free(ck); free(aj); free(ak); free(bb);
    free(row_claim); free(col_claim);
    return any;
}

int or_presolve(const or_lp *lp, const or_settings *s, or_handle **out) {
    or_handle *h = (or_handle *)xcalloc(1, sizeof(or_handle));
    *out = h;
    h->result = RES_UNCHANGED;
    if (!lp || !s) return fail(h, "null argument");
    if (validate_and_copy(h, lp, s)) return 1;
    int32_t m = h->m, n = h->n;

    h->row_on = (uint8_t *)xcalloc((size_t)m, 1);
    h->col_on = (uint8_t *)xcalloc((size_t)n, 1);
    h->col_len = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int32_t i = 0; i < m; ++i) h->row_on[i] = 1;
    for (int32_t j = 0; j < n; ++j) h->col_on[j] = 1;
    for (int64_t k = 0; k < h->nnz; ++k) h->col_len[h->ci[k]]++;
    h->cp = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    h->ri = (int32_t *)xcalloc((size_t)h->nnz + 1, sizeof(int32_t));
    h->cva = (double *)xcalloc((size_t)h->nnz + 1, sizeof(double));
    build_columns(h);
    h->lsrc = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    h->usrc = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int32_t j = 0; j < n; ++j) {
        h->lsrc[j] = isinf(h->lb[j]) ? -1 : -2;
        h->usrc[j] = isinf(h->ub[j]) ? -1 : -2;
    }

    /* round 0: input fixings and crossed bounds / sides */
    h->round = 0;
    int infeasible = 0;
    for (int32_t i = 0; i < m; ++i)
        if (!isinf(h->lhs[i]) && !isinf(h->rhs[i]) && h->lhs[i] > h->rhs[i] + tol_of(s, h->rhs[i]))
            infeasible = 1;
    for (int32_t j = 0; j < n; ++j) {
        double lo = h->lb[j], up = h->ub[j];
        if (isinf(lo) || isinf(up)) continue;
        if (lo > up + tol_of(s, up)) infeasible = 1;
        if (up - lo <= s->fix_tol * mx1(lo)) {
            push(h, REC_FIX_COL, 0, -1, j, -1, lo, h->c[j], 0, 0);
            h->ub[j] = lo;
            h->col_on[j] = 0;
        }
    }
    if (infeasible) { h->result = RES_INFEASIBLE; return 0; }

    int64_t maxlen = 0;
    for (int32_t i = 0; i < m; ++i)
        if (h->rp[i + 1] - h->rp[i] > maxlen) maxlen = h->rp[i + 1] - h->rp[i];
    round_ws w;
    w.lb_s = (double *)xcalloc((size_t)n, sizeof(double));
    w.ub_s = (double *)xcalloc((size_t)n, sizeof(double));
    w.lb_n = (double *)xcalloc((size_t)n, sizeof(double));
    w.ub_n = (double *)xcalloc((size_t)n, sizeof(double));
    w.src_lb = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    w.src_ub = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    w.tmin = (double *)xcalloc((size_t)maxlen, sizeof(double));
    w.tmax = (double *)xcalloc((size_t)maxlen, sizeof(double));
    w.dec = (uint8_t *)xcalloc((size_t)m, 1);
    w.st = (row_stats *)xcalloc((size_t)m, sizeof(row_stats));
    w.down = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    w.up = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    w.pick = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    w.owner = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));

    int stop = 0;
    for (int outer = 0; outer < s->max_outer && !stop; ++outer) {
        for (int r = 0; r < s->max_rounds; ++r) {
            h->round++;
            int changed = run_round(h, &w);
            if (h->result >= RES_INFEASIBLE) { stop = 1; break; }
            if (!changed) break;
        }
        if (stop || (!s->enable_parallel_rows && !s->enable_parallel_cols && !s->enable_doubletons &&
                     !s->enable_dominated))
            break;
        h->round++;
        int merged = s->enable_parallel_rows ? parallel_rows(h) : 0;
        if (h->result >= RES_INFEASIBLE) { stop = 1; break; }
        if (s->enable_parallel_cols) merged |= parallel_cols(h);
        if (s->enable_dominated) {
            merged |= dominated_cols(h);
            if (h->result >= RES_INFEASIBLE) { stop = 1; break; }
        }
        if (s->enable_doubletons) {
            merged |= doubleton_pass(h);
            if (h->result >= RES_INFEASIBLE) { stop = 1; break; }
        }
        if (!merged) break;
    }
    free(w.lb_s); free(w.ub_s); free(w.lb_n); free(w.ub_n);
    free(w.src_lb); free(w.src_ub); free(w.tmin); free(w.tmax); free(w.dec); free(w.st);
    free(w.down); free(w.up); free(w.pick); free(w.owner);

    if (h->result < RES_INFEASIBLE) {
        h->result = h->nrec ? RES_REDUCED : RES_UNCHANGED;
        compact(h);
    }
    return 0;
}

/* Round-1 activities of every row from the input bounds (all columns active);
 * exposed for the pin tests. */
int or_activities(const or_lp *lp, double *minact, double *maxact,
                  int32_t *ninf_min, int32_t *ninf_max) {
    or_handle h;
    memset(&h, 0, sizeof h);
    h.m = lp->m; h.n = lp->n;
    h.rp = (int32_t *)lp->row_ptr; h.ci = (int32_t *)lp->col_idx; h.va = (double *)lp->val;
    h.col_on = (uint8_t *)xcalloc((size_t)lp->n, 1);
    for (int32_t j = 0; j < lp->n; ++j) h.col_on[j] = 1;
    int64_t maxlen = 0;
    for (int32_t i = 0; i < lp->m; ++i)
        if (lp->row_ptr[i + 1] - lp->row_ptr[i] > maxlen) maxlen = lp->row_ptr[i + 1] - lp->row_ptr[i];
    double *tmin = (double *)xcalloc((size_t)maxlen, sizeof(double));
    double *tmax = (double *)xcalloc((size_t)maxlen, sizeof(double));
    for (int32_t i = 0; i < lp->m; ++i) {
        row_stats st;
        compute_stats(&h, i, lp->lb, lp->ub, tmin, tmax, &st);
        minact[i] = st.minact; maxact[i] = st.maxact;
        ninf_min[i] = st.ninf_min; ninf_max[i] = st.ninf_max;
    }
    free(tmin); free(tmax); free(h.col_on);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* postsolve (primal): kept columns from the reduced solution, removed ones   */
/* from their FIX_COL / EMPTY_COL / DUAL_FIX / DOMINATED_COL records         */
/* (constants); then, last record first:                                      */
/*   FREE_SINGLETON  with r = the row's other terms (its original entries,    */
/*       left to right) and s = r clamped to the sides the row had,           */
/*       x_j = (s - r) / a_ij;                                                */
/*   LEADER_BOUNDS   the leader holds the merged value v of its group (the    */
/*       group's PARALLEL_COL records follow it in the same pass); the        */
/*       intervals B_0 = the leader's old bounds, B_s = B_{s-1} + lambda_s    */
/*       [lb_s, ub_s] are rebuilt as presolve built them, and the members,    */
/*       last first, take x_s = the value in [lb_s, ub_s] that keeps          */
/*       v - lambda_s x_s in B_{s-1} (from lb_s if finite, else ub_s, else 0, */
/*       clamped to that range), v -= lambda_s x_s; the leader keeps the rest.*/
/* Every other record keeps the feasible set and leaves x unchanged.          */
/* ------------------------------------------------------------------------- */

static void split_group(const or_handle *h, int64_t t, double *x) {
    const or_record *L = &h->rec[t];
    int32_t k = L->j;
    int64_t e = t + 1;  /* the pass's column records follow */
    while (e < h->nrec && h->rec[e].round == L->round &&
           (h->rec[e].type == REC_PARALLEL_COL || h->rec[e].type == REC_LEADER_BOUNDS)) e++;
    int64_t cnt = 0;
    for (int64_t q = t + 1; q < e; ++q)
        if (h->rec[q].type == REC_PARALLEL_COL && h->rec[q].k == k) cnt++;
    double *blo = (double *)xcalloc((size_t)cnt + 1, sizeof(double));
    double *bup = (double *)xcalloc((size_t)cnt + 1, sizeof(double));
    const or_record **mem = (const or_record **)xcalloc((size_t)cnt + 1, sizeof(or_record *));
    int64_t s = 0;
    blo[0] = L->v[0];
    bup[0] = L->v[1];
    for (int64_t q = t + 1; q < e; ++q) {
        const or_record *r = &h->rec[q];
        if (r->type != REC_PARALLEL_COL || r->k != k) continue;
        mem[s] = r;
        blo[s + 1] = blo[s];
        bup[s + 1] = bup[s];
        add_scaled(h, r->v[0], r->v[1], r->v[2], &blo[s + 1], &bup[s + 1]);
        s++;
    }
    double v = x[k];
    for (int64_t q = cnt - 1; q >= 0; --q) {
        double lam = mem[q]->v[0], l = mem[q]->v[1], u = mem[q]->v[2];
        double a, b;
        if (lam > 0) { a = (v - bup[q]) / lam; b = (v - blo[q]) / lam; }
        else { a = (v - blo[q]) / lam; b = (v - bup[q]) / lam; }
        double lo = a > l ? a : l, hi = b < u ? b : u;
        double pref = !isinf(l) ? l : (!isinf(u) ? u : 0.0);
        double xs = pref < lo ? lo : (pref > hi ? hi : pref);
        x[mem[q]->j] = xs;
        v = v - lam * xs;
    }
    x[k] = v;
    free(blo); free(bup); free(mem);
}

int or_postsolve(const or_handle *h, const double *x_red, double *x) {
    if (h->result >= RES_INFEASIBLE) return 1;
    for (int32_t j = 0; j < h->n; ++j) x[j] = 0.0;
    for (int32_t rj = 0; rj < h->rn; ++rj) x[h->r_colmap[rj]] = x_red[rj];
    for (int64_t t = h->nrec - 1; t >= 0; --t) {
        const or_record *r = &h->rec[t];
        if (r->type == REC_FIX_COL || r->type == REC_EMPTY_COL || r->type == REC_DUAL_FIX ||
            r->type == REC_DOMINATED_COL)
            x[r->j] = r->v[0];
    }
    for (int64_t t = h->nrec - 1; t >= 0; --t) {
        const or_record *r = &h->rec[t];
        if (r->type == REC_LEADER_BOUNDS) {
            split_group(h, t, x);
        } else if (r->type == REC_DOUBLETON_ROW) {
            /* the equality row a_j x_j + a_k x_k = b gives the eliminated x_k */
            x[r->k] = (r->v[2] - r->v[0] * x[r->j]) / r->v[1];
        } else if (r->type == REC_FREE_SINGLETON) {
            double rest = 0.0;
            for (int64_t k = h->rp[r->i]; k < h->rp[r->i + 1]; ++k)
                if (h->ci[k] != r->j) rest = rest + h->va[k] * x[h->ci[k]];
            double side = r->side == 1 ? r->v[1] : r->side == 2 ? r->v[2]
                        : (rest < r->v[1] ? r->v[1] : (rest > r->v[2] ? r->v[2] : rest));
            x[r->j] = (side - rest) / r->v[0];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* postsolve (dual): row duals y[m] and reduced costs z[n] of the original LP */
/* from the reduced problem's row duals y_red (section 2.1, "Postsolver";     */
/* section 3.3 asks for primal and dual solutions of the original problem).   */
/* Convention: c - A'y - z = 0; y_i >= 0 when row i is at lhs, <= 0 at rhs;   */
/* z_j >= 0 when x_j is at lb, <= 0 at ub. The records are undone in reverse  */
/* order:                                                                     */
/*   BOUND_CHANGE  a bound tightened from row k (x_j <= (rhs_k - resmin)/a    */
/*       and the like) that carries a multiplier -- z_j = c_j - a_j'y with    */
/*       that bound's sign -- holds only because row k is at the side that    */
/*       gave it, so the multiplier moves into that row: y_k += z_j / a_kj    */
/*       (then z_j = 0). The other columns of row k are then at the bounds    */
/*       the residual activity used, which are their bounds before this       */
/*       round: a reduced cost this induces is carried by the next earlier    */
/*       tightening of that bound, reached later in the reverse pass (a       */
/*       chain of rounds is followed back to the original bounds). A bound    */
/*       superseded by a later tightening has z_j = 0 by then.                */
/*   LEADER_SIDES  the merged side of a parallel-row leader L that is active  */
/*       (y_L > 0: lhs, y_L < 0: rhs) is the side of the row r that gave it,  */
/*       with a_r = lambda_r a_L: y_r = y_L / lambda_r and y_L = 0.           */
/*   every other record leaves y: rows removed as empty, redundant or         */
/*       singleton start at y = 0 (a singleton's bounds reach it through the  */
/*       bound changes it sourced), fixed, empty and dual-fixed columns take  */
/*       their reduced cost from z = c - A'y (a dual-fixed column has no      */
/*       locks towards its bound, so the active rows' multipliers can only    */
/*       push z_j further to that bound's sign).                              */
/*   FREE_SINGLETON  the row's dual is y_i = c_j / a_ij (z_j = 0 for the free */
/*       column), set before the pass: after the substitution every other    */
/*       column of the row costs c_k - y_i a_ik, so the reduced costs that   */
/*       later records read already hold the row's share.                     */
/* Every z_j = c_j - sum_i a_ij y_i is summed over the column's rows in      */
/* ascending order, left to right.                                            */
/* ------------------------------------------------------------------------- */

static double col_red_cost(const or_handle *h, const int32_t *cp, const int32_t *ri, const double *cva,
                           const double *y, int32_t j) {
    double s = 0.0;
    for (int32_t q = cp[j]; q < cp[j + 1]; ++q) s = s + cva[q] * y[ri[q]];
    return h->c0[j] - s;
}

/* The dual a doubleton substitution gives its row (r = the DOUBLETON_ROW
 * record): with x_k between its bounds, z_k = c_k - a_k'y = 0, i.e.
 * (c_k - sum over the input's column k of a_rk y_r, row i left out) / a_ik,
 * c_k the cost x_k had then. Column k's entries were never rewritten before
 * (only kept columns are), so the input's column is the one of that time. */
static double doubleton_dual(const int32_t *cp, const int32_t *ri, const double *cva, const double *y,
                             const or_record *r) {
    double ay = 0.0;
    for (int32_t q = cp[r->k]; q < cp[r->k + 1]; ++q)
        if (ri[q] != r->i) ay = ay + cva[q] * y[ri[q]];
    return (r->v[3] - ay) / r->v[1];
}

/* Reduced cost of column j in the problem of the time being undone: the
 * input's column j, and, while the substitution that kept j is not undone
 * yet, its rows carry the row's multiplier too (each rewritten row r is
 * r - f_r row_i, and the cost c_j - (c_k/a_k) a_j): z_j - a_ij * (that
 * row's dual as the substitution would give it now). */
static double cur_red_cost(const or_handle *h, const int32_t *cp, const int32_t *ri, const double *cva,
                           const double *y, const int64_t *pending, int32_t j) {
    double z = col_red_cost(h, cp, ri, cva, y, j);
    if (pending[j] >= 0) {
        const or_record *r = &h->rec[pending[j]];
        z = z - r->v[0] * doubleton_dual(cp, ri, cva, y, r);
    }
    return z;
}

int or_postsolve_dual(const or_handle *h, const double *x_red, const double *y_red,
                      double *x, double *y, double *z) {
    if (h->result >= RES_INFEASIBLE) return 1;
    if (or_postsolve(h, x_red, x)) return 1;
    int32_t m = h->m, n = h->n;
    for (int32_t i = 0; i < m; ++i) y[i] = 0.0;
    for (int32_t ri0 = 0; ri0 < h->rm; ++ri0) y[h->r_rowmap[ri0]] = y_red[ri0];
    /* the original matrix by columns (rows ascending within a column) */
    int32_t *cp = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    int32_t *ri = (int32_t *)xcalloc((size_t)h->nnz, sizeof(int32_t));
    double *cva = (double *)xcalloc((size_t)h->nnz, sizeof(double));
    for (int64_t k = 0; k < h->nnz; ++k) cp[h->ci0[k] + 1]++;
    for (int32_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
    int32_t *fill = (int32_t *)xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int32_t j = 0; j < n; ++j) fill[j] = cp[j];
    for (int32_t i = 0; i < m; ++i)
        for (int32_t k = h->rp[i]; k < h->rp[i + 1]; ++k) {
            int32_t q = fill[h->ci0[k]]++;
            ri[q] = i;
            cva[q] = h->va0[k];
        }
    /* lambda of every row removed as parallel (a_r = lambda a_leader); the
     * doubleton substitution that kept each column, not undone yet */
    double *lam = (double *)xcalloc((size_t)m + 1, sizeof(double));
    int64_t *pending = (int64_t *)xcalloc((size_t)n + 1, sizeof(int64_t));
    for (int32_t j = 0; j < n; ++j) pending[j] = -1;
    for (int64_t t = 0; t < h->nrec; ++t) {
        if (h->rec[t].type == REC_PARALLEL_ROW) lam[h->rec[t].i] = h->rec[t].v[0];
        if (h->rec[t].type == REC_DOUBLETON_ROW) pending[h->rec[t].j] = t;
        /* a row substituted into the objective has the dual c_j / a_ij from
         * the moment it leaves: the costs the later problems carry are
         * c_k - y_i a_ik, so the reduced costs read while undoing them see it */
        if (h->rec[t].type == REC_FREE_SINGLETON) y[h->rec[t].i] = h->rec[t].v[3] / h->rec[t].v[0];
    }
    for (int64_t t = h->nrec - 1; t >= 0; --t) {
        const or_record *r = &h->rec[t];
        if (r->type == REC_BOUND_CHANGE) {
            int32_t j = r->j, k = r->k;
            if (k < 0) continue;
            double zj = cur_red_cost(h, cp, ri, cva, y, pending, j);
            if ((r->side == 0 && zj > 0.0) || (r->side == 1 && zj < 0.0)) y[k] = y[k] + zj / r->v[2];
        } else if (r->type == REC_FREE_SINGLETON) {
            /* the substituted column is free: z_j = 0 gives the row's dual */
            y[r->i] = r->v[3] / r->v[0];
        } else if (r->type == REC_DOUBLETON_ROW) {
            /* the row's dual: the part that makes z_k = 0, added to what a
             * binding bound moved from x_k to x_j gave it (undone just before;
             * then z_j = 0 and x_k sits at its bound) */
            y[r->i] = y[r->i] + doubleton_dual(cp, ri, cva, y, r);
            pending[r->j] = -1;
        } else if (r->type == REC_LEADER_SIDES) {
            int32_t L = r->i;
            double yl = y[L];
            int32_t src = yl > 0.0 ? r->j : (yl < 0.0 ? r->k : -1);
            if (src >= 0 && src != L) {
                y[src] = yl / lam[src];
                y[L] = 0.0;
            }
        }
    }
    for (int32_t j = 0; j < n; ++j) z[j] = col_red_cost(h, cp, ri, cva, y, j);
    free(cp); free(ri); free(cva); free(fill); free(lam); free(pending);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* accessors                                                                  */
/* ------------------------------------------------------------------------- */

void or_free(or_handle *h) {
    if (!h) return;
    free(h->rp); free(h->ci); free(h->va); free(h->lhs); free(h->rhs);
    free(h->lb); free(h->ub); free(h->c); free(h->c0); free(h->row_on); free(h->col_on); free(h->lsrc); free(h->usrc);
    free(h->ci0); free(h->va0); free(h->col_mod);
    free(h->cp); free(h->ri); free(h->cva);
    free(h->col_len); free(h->rec);
    free(h->r_rp); free(h->r_ci); free(h->r_va); free(h->r_cp); free(h->r_ri); free(h->r_cva);
    free(h->r_lhs); free(h->r_rhs); free(h->r_lb); free(h->r_ub); free(h->r_c);
    free(h->r_rowmap); free(h->r_colmap); free(h->r_rcls); free(h->r_ccls);
    free(h);
}

const char *or_error(const or_handle *h) { return h ? h->err : "null handle"; }
int32_t or_result(const or_handle *h) { return h->result; }
int32_t or_rounds(const or_handle *h) { return h->round; }
int64_t or_num_records(const or_handle *h) { return h->nrec; }
const or_record *or_records(const or_handle *h) { return h->rec; }

void or_reduced_dims(const or_handle *h, int32_t *m, int32_t *n, int64_t *nnz, double *obj_offset) {
    *m = h->rm; *n = h->rn; *nnz = h->rnnz; *obj_offset = h->roff;
}

void or_reduced_copy(const or_handle *h, int32_t *row_ptr, int32_t *col_idx, double *val,
                     int32_t *col_ptr, int32_t *row_idx, double *cval,
                     double *lhs, double *rhs, double *lb, double *ub, double *c,
                     int32_t *row_map, int32_t *col_map,
                     uint8_t *row_class, uint8_t *col_class) {
    memcpy(row_ptr, h->r_rp, ((size_t)h->rm + 1) * sizeof(int32_t));
    memcpy(col_ptr, h->r_cp, ((size_t)h->rn + 1) * sizeof(int32_t));
    if (h->rnnz) {
        memcpy(col_idx, h->r_ci, (size_t)h->rnnz * sizeof(int32_t));
        memcpy(val, h->r_va, (size_t)h->rnnz * sizeof(double));
        memcpy(row_idx, h->r_ri, (size_t)h->rnnz * sizeof(int32_t));
        memcpy(cval, h->r_cva, (size_t)h->rnnz * sizeof(double));
    }
    if (h->rm) {
        memcpy(lhs, h->r_lhs, (size_t)h->rm * sizeof(double));
        memcpy(rhs, h->r_rhs, (size_t)h->rm * sizeof(double));
        memcpy(row_map, h->r_rowmap, (size_t)h->rm * sizeof(int32_t));
        memcpy(row_class, h->r_rcls, (size_t)h->rm);
    }
    if (h->rn) {
        memcpy(lb, h->r_lb, (size_t)h->rn * sizeof(double));
        memcpy(ub, h->r_ub, (size_t)h->rn * sizeof(double));
        memcpy(c, h->r_c, (size_t)h->rn * sizeof(double));
        memcpy(col_map, h->r_colmap, (size_t)h->rn * sizeof(int32_t));
        memcpy(col_class, h->r_ccls, (size_t)h->rn);
    }
}
