/*
 * psl_oracle.h -- sequential CPU reference presolver (TEST INFRASTRUCTURE).
 *
 * This oracle exists only to check the GPU library. It is plain, slow and
 * sequential: every loop runs in ascending index order and every sum is the
 * canonical pairwise tree written out recursively. It shares no code, header,
 * constant table or helper with the GPU library; both were written separately
 * from the same reading of the paper (Cederberg & Boyd, "GPU-Accelerated
 * Presolving for Linear Programming"). Only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Problem form: eq. (1), section 2.1:
 *     minimize c'x + obj_offset  s.t.  lhs <= A x <= rhs,  lb <= x <= ub.
 */
#ifndef PSL_ORACLE_H
#define PSL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int32_t *row_ptr, *col_idx;
    const double *val;
    const double *lhs, *rhs, *lb, *ub, *c;
    double obj_offset;
} or_lp;

typedef struct {
    int32_t max_rounds, max_outer, enable_parallel_rows;
    double feas_tol, fix_tol, min_improve, par_tol, inf_value, coef_tol;
    int32_t enable_dual_fix;  /* 1: lock-based dual fixing in every round */
    int32_t enable_free_singletons;  /* 1: zero-cost free column singletons */
    int32_t enable_parallel_cols;    /* 1: parallel columns in the parallel pass */
    int32_t enable_forcing_rows;     /* 1: forcing rows in every round */
    int32_t enable_doubletons;       /* 1: doubleton-equality substitution pass */
    int32_t enable_dominated;        /* 1: dominated columns (implied dual bounds) pass */
} or_settings;

/* 48-byte postsolve record; the field meaning per type is listed in the .c */
typedef struct {
    uint8_t type, side;
    uint16_t round;
    int32_t i, j, k;
    double v[4];
} or_record;

typedef struct or_handle or_handle;

/* status: 0 ok, 1 invalid input / settings */
int or_presolve(const or_lp *lp, const or_settings *s, or_handle **out);
void or_free(or_handle *h);
const char *or_error(const or_handle *h);

/* result: 0 reduced, 1 unchanged, 2 infeasible, 3 unbounded or infeasible */
int32_t or_result(const or_handle *h);
int32_t or_rounds(const or_handle *h);
int64_t or_num_records(const or_handle *h);
const or_record *or_records(const or_handle *h);

/* reduced problem (valid for results 0 and 1) */
void or_reduced_dims(const or_handle *h, int32_t *m, int32_t *n, int64_t *nnz, double *obj_offset);
void or_reduced_copy(const or_handle *h, int32_t *row_ptr, int32_t *col_idx, double *val,
                     int32_t *col_ptr, int32_t *row_idx, double *cval,
                     double *lhs, double *rhs, double *lb, double *ub, double *c,
                     int32_t *row_map, int32_t *col_map,
                     uint8_t *row_class, uint8_t *col_class);

/* primal postsolve: x_red[n_red] -> x[n] */
int or_postsolve(const or_handle *h, const double *x_red, double *x);

/* primal and dual postsolve: x_red[n_red], y_red[m_red] (row duals of the
 * reduced problem) -> x[n], y[m], z[n] (z = c - A'y); convention and rules in
 * the .c */
int or_postsolve_dual(const or_handle *h, const double *x_red, const double *y_red,
                      double *x, double *y, double *z);

/* stand-alone pieces exposed for the pin tests */
double or_pairwise_sum(const double *x, int64_t len);
uint64_t or_row_key(const int32_t *cols, const double *vals, int64_t len);
int or_activities(const or_lp *lp, double *minact, double *maxact,
                  int32_t *ninf_min, int32_t *ninf_max);

#ifdef __cplusplus
}
#endif
#endif
