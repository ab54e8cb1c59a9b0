/*
 * psl.h -- C-ABI of libpsl, a GPU (MI355X, gfx950) presolve sweep for linear
 * programs of the form of eq. (1) in section 2.1 of Cederberg & Boyd,
 * "GPU-Accelerated Presolving for Linear Programming":
 *
 *     minimize c'x + obj_offset   s.t.   lhs <= A x <= rhs,   lb <= x <= ub.
 *
 * One call to psl_presolve_run performs, in rounds, the reductions of
 * sections 3.1 and 3.2 of that paper that are data parallel over rows and
 * columns (activities, bound tightening, empty / redundant / singleton rows,
 * fixed and empty columns, parallel rows), then emits a reduced LP of the same
 * form (section 3.3) and a stream of postsolve records (section 2.1,
 * "Postsolver"). All of it runs in the library's HIP kernels; postsolve runs on
 * the host, as in section 3.3.
 *
 * Conventions for every function:
 *   - The return value is a psl_status. On any status other than PSL_OK the
 *     out-parameters are left untouched and psl_last_error() describes the
 *     failure (per handle; NULL handle -> the last create error of the thread).
 *   - Infeasible or unbounded problems are results (psl_result), not errors.
 *   - Arrays are plain pointers with explicit sizes. Where a struct carries a
 *     psl_mem field, PSL_MEM_HOST means host memory and PSL_MEM_DEVICE means
 *     memory of the device named in psl_settings.device.
 *   - All device work is ordered on psl_settings.stream (a hipStream_t, or
 *     NULL for the default stream). Calls return after that work is complete
 *     unless stated otherwise.
 *   - Infinity: a side or bound whose magnitude is >= inf_value (default 1e20),
 *     or +-INFINITY, is infinite.
 *   - One handle must not be used from two threads at once.
 */
#ifndef PSL_H
#define PSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSL_OK = 0,
    PSL_ERR_INVALID = 1,     /* malformed input, bad argument or settings      */
    PSL_ERR_OOM = 2,         /* device or host allocation failed               */
    PSL_ERR_DEVICE = 3,      /* a HIP call failed                              */
    PSL_ERR_STATE = 4,       /* call not valid in the handle's current state   */
    PSL_ERR_CAPACITY = 5,    /* a size limit of the library was exceeded       */
    PSL_ERR_UNSUPPORTED = 6  /* feature not provided (e.g. dual postsolve of a
                                server ticket)                                 */
} psl_status;

typedef enum {
    PSL_RES_REDUCED = 0,                 /* at least one reduction applied      */
    PSL_RES_UNCHANGED = 1,               /* no reduction found                  */
    PSL_RES_INFEASIBLE = 2,              /* a row or column is infeasible       */
    PSL_RES_UNBOUNDED_OR_INFEASIBLE = 3  /* an empty column with a cost that
                                            points to an infinite bound         */
} psl_result;

typedef enum { PSL_MEM_HOST = 0, PSL_MEM_DEVICE = 1 } psl_mem;

/* The input LP, eq. (1). CSR with int32 indices: row_ptr[m+1] (row_ptr[0] = 0,
 * non-decreasing, row_ptr[m] = nnz), col_idx[nnz] strictly ascending within
 * each row and in [0, n), val[nnz] finite and non-zero. lhs/rhs[m], lb/ub/c[n].
 * lhs must not be +inf, rhs not -inf; lb not +inf, ub not -inf; no NaN.
 * m, n and nnz < 2^30 (so that sums of row and column counts, and twice
 * either, stay within int32 on the device). The library copies everything
 * at create/reload: the caller keeps ownership of these arrays and may free
 * them once the call returns. */
typedef struct {
    int32_t m, n;
    int64_t nnz;
    psl_mem mem;
    const int32_t *row_ptr, *col_idx;
    const double *val;
    const double *lhs, *rhs, *lb, *ub, *c;
    double obj_offset;
} psl_lp;

/* Settings. The tolerances are part of the round semantics: changing them
 * changes which reductions fire. Defaults from psl_settings_default():
 *   max_rounds 16, max_outer 4, enable_parallel_rows 1,
 *   feas_tol 1e-9, fix_tol 1e-9, min_improve 1e-7, par_tol 1e-9,
 *   inf_value 1e20, coef_tol 1e-9, bin thresholds from the tuner (NULL),
 *   device 0, stream NULL, split_sweep 0, enable_dual_fix 0,
 *   enable_free_singletons 0, enable_parallel_cols 0, enable_forcing_rows 0,
 *   enable_doubletons 0.
 * bin_thresholds (optional, n_bins = 2 or 3): [0] the longest row swept by one
 * 64-lane wavefront (16..512, default 512); [1] positions per workgroup chunk
 * of longer rows (a power of two >= 2048, default 2048); [2] the longest row
 * swept by an 8-lane group (8, the default, or 4: rows of 5..8 entries then go
 * to 16-lane groups). They change only the speed, never a result; psl_tune
 * picks them by timing. */
typedef struct {
    int32_t max_rounds;            /* propagation rounds per outer cycle        */
    int32_t max_outer;             /* outer cycles (rounds, then parallel rows) */
    int32_t enable_parallel_rows;
    double feas_tol;               /* tol(s) = feas_tol * max(1, |s|)           */
    double fix_tol;                /* fix when ub - lb <= fix_tol*max(1,|lb|)   */
    double min_improve;            /* accept a bound if it improves by more
                                      than min_improve * max(1, |bound|)        */
    double par_tol;                /* parallel-row coefficient tolerance        */
    double inf_value;
    double coef_tol;               /* |a| below this gives no implied bound     */
    const int32_t *bin_thresholds;
    int32_t n_bins;
    int32_t device;
    void *stream;                  /* hipStream_t or NULL                       */
    int32_t split_sweep;           /* 0: one row-sweep launch per round; 1: three
                                      (short rows, wavefront rows, long-row
                                      chunks). Speed only, never a result.     */
    int32_t enable_dual_fix;       /* 1: dual fixing in every round (a dual
                                      explorer, section 2.1, on variable locks,
                                      section 3.2): after the round's row
                                      removals, a column with no alive row
                                      keeping it from moving towards the bound
                                      its cost prefers (c > 0: down, c < 0: up,
                                      c = 0: either, a finite bound, lower
                                      first) is fixed there (DUAL_FIX); such a
                                      bound at infinity gives
                                      PSL_RES_UNBOUNDED_OR_INFEASIBLE. Keeps an
                                      optimal solution, not the feasible set.
                                      0 (default) or 1.                        */
    int32_t enable_free_singletons;/* 1: at the end of every round, a column
                                      in one alive row i, whose bounds are
                                      infinite or were tightened only from
                                      row i (implied by it), leaves with row i
                                      (FREE_SINGLETON, section 3.2 "Column
                                      singletons"); the lowest such column of
                                      a row goes. A column with a cost is
                                      substituted into the objective: with
                                      r = c_j / a_ij the row goes to its lhs
                                      (r > 0) or rhs (r < 0; infinite:
                                      PSL_RES_UNBOUNDED_OR_INFEASIBLE), the
                                      row's other costs become c_k - r a_ik,
                                      the offset gains r * side; rows sharing
                                      a column then take turns, lowest first.
                                      Postsolve takes x_j from the row, and
                                      the row's dual is r. 0 (default) or 1.   */
    int32_t enable_parallel_cols;  /* 1: after the parallel rows, parallel
                                      columns (section 3.2, "Parallel
                                      columns": parallel rows of [c A'] over
                                      the alive rows, columns of any length)
                                      merge into the
                                      first column of their group, whose
                                      interval becomes the sum of the scaled
                                      intervals (in column order; a group
                                      whose sum reaches a lower bound of +inf
                                      or an upper bound of -inf, |v| >=
                                      inf_value, is not merged);
                                      PARALLEL_COL / LEADER_BOUNDS. 0 (default)
                                      or 1. The parallel pass runs when either
                                      this or enable_parallel_rows is set.     */
    int32_t enable_forcing_rows;   /* 1: forcing rows in every round (a primal
                                      explorer, section 2.1): a row with at
                                      least two active columns whose finite min
                                      activity reaches its rhs within feas_tol
                                      (or max activity its lhs) leaves
                                      (FORCING_ROW), and every active column is
                                      fixed at the bound giving that activity
                                      (its other bound becomes a candidate of
                                      the round, so the column decisions fix
                                      it). Rows with an active |a| < coef_tol
                                      are not forcing. 0 (default) or 1.       */
    int32_t enable_doubletons;     /* 1: doubleton-equality substitution (the
                                      doubleton-row explorer, section 2.1) once
                                      per outer cycle after the parallel
                                      passes: an alive row with lhs = rhs and
                                      two active columns eliminates one,
                                      x_k = (b - a_j x_j) / a_k, from its other
                                      rows (fill-in on column j, rows rewritten
                                      in place), costs and bounds; rows sharing
                                      a column take turns, lowest first; a
                                      column kept by a substitution takes part
                                      in no other (DOUBLETON_ROW). 0 (default)
                                      or 1.                                    */
    int64_t device_records;        /* the postsolve stack (section 3.3): 0
                                      (default) lets the device record buffer
                                      grow as a run needs it; R > 0 keeps a
                                      fixed device stack of R records that is
                                      flushed to host memory (and emptied)
                                      whenever the next phase's records might
                                      not fit. R must hold one phase's worst
                                      case, the larger of m + 3n + 16 (a
                                      round) and m + n + 16 (a parallel pass)
                                      plus n with enable_dominated and m + 2n
                                      with enable_doubletons, else
                                      PSL_ERR_INVALID at create. Single-LP
                                      presolvers only (batches and servers:
                                      PSL_ERR_UNSUPPORTED); not with
                                      psl_presolve_noalloc. Records, reduced
                                      problem and postsolve are the same.     */
    int32_t enable_dominated;      /* 1: dominated columns once per outer cycle
                                      after the parallel columns (a dual
                                      explorer, section 2.1): row duals are
                                      bounded by the sides' signs and by column
                                      singletons (no upper bound: z >= 0, no
                                      lower bound: z <= 0); a column whose
                                      reduced cost is then above feas_tol *
                                      max(1, |c|) for every such dual is fixed
                                      at its lower bound, below the negative
                                      tolerance at its upper bound
                                      (DOMINATED_COL; an infinite one, or
                                      crossing dual bounds: unbounded or
                                      infeasible). 0 (default) or 1.           */
} psl_settings;

/* Postsolve record: 48 bytes, emitted in the order (round, phase, index,
 * side). Unused integer fields are -1, unused doubles 0.
 *   type 1 FIX_COL        j; v = {value, c_j}
 *   type 2 EMPTY_COL      j; v = {value, c_j}
 *   type 3 EMPTY_ROW      i; v = {activity, lhs, rhs}
 *   type 4 REDUNDANT_ROW  i; v = {min activity or -inf, max activity or +inf,
 *                                 lhs, rhs}
 *   type 5 SINGLETON_ROW  i, j = its active column; v = {a_ij, lhs, rhs}
 *   type 6 BOUND_CHANGE   j, side (0 lower, 1 upper), k = source row;
 *                         v = {old bound, new bound, a_kj}
 *   type 7 PARALLEL_ROW   i = removed row, k = leader; v = {lambda, lhs, rhs}
 *   type 8 LEADER_SIDES   i = leader, j = row giving lhs, k = row giving rhs;
 *                         v = {old lhs, old rhs, new lhs, new rhs}
 *   type 9 DUAL_FIX       j, side (0 at its lower, 1 at its upper bound);
 *                         v = {value, c_j} (only with enable_dual_fix)
 *   type 10 FREE_SINGLETON i = removed row, j = its (implied) free column;
 *                         side 0: c_j = 0, 1: the row went to its lhs, 2: to
 *                         its rhs; v = {a_ij, lhs_i, rhs_i, c_j} (the values
 *                         then; only with enable_free_singletons)
 *   type 11 PARALLEL_COL  j = merged column, k = its leader;
 *                         v = {lambda (a_j = lambda a_k), lb_j, ub_j}
 *   type 12 LEADER_BOUNDS j = leader; v = {old lb, old ub, new lb, new ub}
 *                         (both only with enable_parallel_cols; a leader's
 *                         record precedes its group's PARALLEL_COL records)
 *   type 13 FORCING_ROW   i; side 0: the min activity reached rhs, 1: the
 *                         max activity reached lhs; v = {that activity, lhs,
 *                         rhs} (only with enable_forcing_rows; its columns'
 *                         BOUND_CHANGE and FIX_COL records follow in the same
 *                         round)
 *   type 14 DOUBLETON_ROW i = the equality row, j = the kept column, k = the
 *                         eliminated one; v = {a_ij, a_ik, b, c_k then}, b the
 *                         row's side less its removed columns' constant (only
 *                         with enable_doubletons; the bounds it moves to x_j
 *                         follow as BOUND_CHANGE records from row i)
 *   type 15 DOMINATED_COL j, side 0 (at its lower bound) or 1 (upper);
 *                         v = {value, c_j} (only with enable_dominated)
 * round 0 holds input fixings; each propagation round and each parallel-row
 * pass has its own round number. */
typedef struct {
    uint8_t type, side;
    uint16_t round;
    int32_t i, j, k;
    double v[4];
} psl_record;

typedef struct {
    int32_t rounds;                /* last round number used                    */
    int32_t outer_cycles;
    int64_t records;
    int64_t nnz_in, nnz_out;
    int32_t m_out, n_out;
    /* device time per phase (ms), measured with HIP events on the stream */
    double ms_ingest, ms_sweep, ms_decide, ms_parallel, ms_compact, ms_total;
    int64_t sweep_launches;        /* launches of the row-sweep kernel          */
    double sweep_bytes;            /* algorithmic bytes of those launches       */
    double ms_long;                /* long-row chunk statistics (before each
                                      sweep launch)                             */
    double alg_bytes;              /* algorithmic (compulsory) HBM bytes of
                                      every pass of the run: per round the
                                      sweep (12 B per swept nonzero, 48 B per
                                      swept row, 32 B per column it can touch)
                                      and the decisions (40 B per row and
                                      column, 48 B per record); per parallel
                                      pass 40 B per row, 12 B per nonzero and
                                      the records; compaction 12 B per input
                                      and 24 B per reduced nonzero, 32 B per
                                      reduced row, 40 B per reduced column     */
    double ingest_bytes;           /* the same for the ingest of the LP (create
                                      or reload): 36 B per nonzero (read, copy,
                                      transposed copy), 32 B per row, 48 B per
                                      column                                    */
    int64_t sweep_nnz;             /* nonzeros swept by those launches (each
                                      gathers its column's bounds once)         */
    int64_t record_flushes;        /* flushes of the device record stack to
                                      host memory (device_records > 0)          */
} psl_stats;

/* The reduced problem. DEVICE pointers owned by the handle, valid until the
 * next psl_presolve_run / psl_presolve_reload or psl_presolve_free.
 * row_map / col_map give the original index of each kept row / column.
 * row_class: 0 other, 1 singleton, 2 doubleton equality, 3 doubleton
 * inequality. col_class: 0 other, 1 free singleton, 2 singleton, 3 doubleton.
 * Rows and columns of these classes are detected and listed, not eliminated. */
typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int32_t *row_ptr, *col_idx;
    const double *val;
    const int32_t *col_ptr, *row_idx;
    const double *cval;
    const double *lhs, *rhs, *lb, *ub, *c;
    double obj_offset;
    const int32_t *row_map, *col_map;
    const uint8_t *row_class, *col_class;
} psl_reduced_view;

typedef struct psl_presolver psl_presolver;

/* Fill *s with the defaults listed above. */
void psl_settings_default(psl_settings *s);

/* Validate and copy the LP to the device (section 3.2, "Internal data
 * structures": A is kept with its transpose; sizes and flags are the state).
 * Settings are copied. Errors: PSL_ERR_INVALID for malformed input (the
 * checks listed at psl_lp) or settings, PSL_ERR_OOM, PSL_ERR_DEVICE. */
psl_status psl_presolve_create(const psl_lp *lp, const psl_settings *s, psl_presolver **out);

/* Replace the handle's LP with another one of the same m, n and nnz, reusing
 * its device memory (no allocation). Same checks as create. */
psl_status psl_presolve_reload(psl_presolver *p, const psl_lp *lp);

/* Run the sweep: rounds of activities + bound tightening + row/column
 * reductions (section 3.1, "Bound tightening"), parallel rows (section 3.2),
 * then compaction. Writes the outcome to *res and, if stats is non-NULL,
 * statistics. Errors: PSL_ERR_STATE if already run since create/reload,
 * PSL_ERR_DEVICE, PSL_ERR_OOM. */
psl_status psl_presolve_run(psl_presolver *p, psl_result *res, psl_stats *stats);

/* View of the reduced problem (section 3.3: the presolver emits a reduced LP
 * of the same form as the input, kept rows by kept columns in their original
 * order, sides shifted by the removed columns' constants, the removed
 * columns' costs in the objective offset; device pointers owned by the
 * handle, valid until the next run, reload or free). PSL_ERR_STATE unless the
 * last run gave PSL_RES_REDUCED or PSL_RES_UNCHANGED. */
psl_status psl_reduced_problem(const psl_presolver *p, psl_reduced_view *out);

/* Number of postsolve records of the last run, and a copy of them into the
 * HOST array out[cap] (cap >= count, else PSL_ERR_CAPACITY). */
psl_status psl_records(const psl_presolver *p, int64_t *count, psl_record *out, int64_t cap);

/* Postsolve on the host (section 2.1, "Postsolver"; section 3.3 asks for the
 * primal and dual solutions of the original problem). All arrays are HOST
 * memory.
 *   Primal: x_red[n_red] -> x[n]. Kept columns come from x_red, removed
 *   columns from their FIX_COL / EMPTY_COL / DUAL_FIX records; then, last
 *   record first, a FREE_SINGLETON column from its row: with rest = the
 *   row's other terms (its original entries, left to right) and s = the
 *   recorded side (side 1: lhs, 2: rhs) or, for side 0, rest clamped to the
 *   recorded sides, x_j = (s - rest) / a_ij (the original rows are read back
 *   from the device); a LEADER_BOUNDS group splits its
 *   leader's merged value v: with B_0 = the old leader bounds and B_s =
 *   B_{s-1} + lambda_s [lb_s, ub_s] rebuilt in member order, members, last
 *   first, take the value in [lb_s, ub_s] keeping v - lambda_s x_s in
 *   B_{s-1} (from lb_s if finite, else ub_s, else 0, clamped), v -= lambda_s
 *   x_s, and the leader keeps the rest. The other record types keep the
 *   feasible set and leave x unchanged.
 *   Dual (when y_red != NULL): the reduced problem's row duals y_red[m_red]
 *   -> row duals y[m] and reduced costs z[n] of the original LP, with the
 *   convention c - A'y - z = 0, y_i >= 0 at lhs and <= 0 at rhs, z_j >= 0 at
 *   lb and <= 0 at ub. Kept rows take y_red, other rows start at 0, and the
 *   records are undone last to first: a BOUND_CHANGE with a source row k whose
 *   column carries a multiplier of that bound's sign (z_j > 0 for a lower,
 *   < 0 for an upper bound) moves it into row k (y_k += z_j / a_kj); a
 *   LEADER_SIDES record whose leader L has an active merged side (y_L > 0:
 *   lhs, < 0: rhs) moves y_L to the row r that gave that side
 *   (y_r = y_L / lambda_r, y_L = 0); a FREE_SINGLETON row takes
 *   y_i = c_j / a_ij (recorded values); the other records keep y. Then
 *   z = c - A'y, each a_j'y summed over column j's rows in ascending order,
 *   left to right. The original matrix is read back from the device.
 *   z_red is accepted and not read (the reduced costs follow from y); y and
 *   z are written only when y_red is given. */
psl_status psl_postsolve(psl_presolver *p, const double *x_red, const double *y_red,
                         const double *z_red, double *x, double *y, double *z);

void psl_presolve_free(psl_presolver *p);

/* Message of the last failure on p (or of the last failed create when p is
 * NULL). Never NULL. */
const char *psl_last_error(const psl_presolver *p);

/* ---- Presolve without allocation --------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture
 * of the surrounding work, tight serving loops, harnesses that forbid
 * hipMalloc. psl_presolve_noalloc performs the same presolve as
 * psl_presolve_create + psl_presolve_run (identical outcome, records and
 * reduced problem) but keeps all of its device working memory (the copy of
 * the LP and its transpose, round state, bins, candidates, records, the
 * reduced problem before it is copied out) in one static device array of
 * PSL_NOALLOC_SCRATCH_BYTES per device, which the library's code object
 * reserves when it is loaded on a device and holds until the process ends.
 * A call allocates and frees no device memory and no pinned host memory;
 * its host-side bookkeeping uses the ordinary C++ heap. */
#define PSL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* Caller-owned DEVICE buffers for the results, sized for the INPUT LP (the
 * reduced problem is never larger), and the sizes written on PSL_OK. */
typedef struct {
    int32_t *row_ptr;              /* [m + 1] reduced CSR                        */
    int32_t *col_idx;              /* [nnz]                                      */
    double *val;                   /* [nnz]                                      */
    int32_t *col_ptr;              /* [n + 1] reduced transposed copy            */
    int32_t *row_idx;              /* [nnz]                                      */
    double *cval;                  /* [nnz]                                      */
    double *lhs, *rhs;             /* [m]                                        */
    double *lb, *ub, *c;           /* [n]                                        */
    int32_t *row_map;              /* [m] reduced -> original row                */
    int32_t *col_map;              /* [n] reduced -> original column             */
    uint8_t *row_class;            /* [m] as in psl_reduced_view                 */
    uint8_t *col_class;            /* [n]                                        */
    psl_record *records;           /* [records_cap] postsolve records            */
    int64_t records_cap;
    /* outputs */
    int32_t m_out, n_out;          /* reduced sizes (0 when infeasible or
                                      unbounded: no reduced problem)             */
    int64_t nnz_out;
    double obj_offset;
    int64_t records_out;           /* records written                            */
} psl_noalloc_out;

/* Presolve lp (host or device arrays, checked as at psl_presolve_create) with
 * settings s (NULL: defaults; the stream orders all device work, and the call
 * returns when it is complete) in the static scratch of device s->device, and
 * copy the reduced problem and the records into out's buffers. The scratch
 * set-up (its device address, the timing events) is done once per device, at
 * the first call on it.
 * Errors: PSL_ERR_INVALID (null arguments or output buffers, invalid LP or
 * settings), PSL_ERR_CAPACITY (the LP's working set exceeds
 * PSL_NOALLOC_SCRATCH_BYTES -- about 250 bytes per nonzero plus about 200 per
 * row and column -- or its records exceed records_cap or the scratch left for
 * them), PSL_ERR_DEVICE. The message is psl_last_error(NULL) on the calling
 * thread. out's outputs are written only on PSL_OK.
 * Concurrency: every call on one device uses that device's scratch, which
 * keeps the last call's contents (a call clears the part it uses before
 * reading it). The library takes a per-device lock for the whole call, so
 * calls from several threads on one device run one after another; without
 * that lock two overlapping calls on one GPU would race on the scratch. */
psl_status psl_presolve_noalloc(const psl_lp *lp, const psl_settings *s, psl_noalloc_out *out, psl_result *res,
                                psl_stats *stats);

/* ---- Autotuning -------------------------------------------------------------
 * The launch shapes (bin thresholds, one or three sweep launches) change only
 * the speed. psl_tune times presolves of the given LPs (one batch when k > 1)
 * under candidate shapes and reports the fastest; every candidate must give
 * the same outcome and record count as the first (else PSL_ERR_DEVICE). */
typedef struct {
    int32_t bin_thresholds[3];     /* fastest: as psl_settings.bin_thresholds   */
    int32_t split_sweep;           /* fastest launch split                       */
    int32_t candidates;            /* shapes timed                               */
    double ms_best;                /* device ms of a presolve (fastest rep), fastest */
    double ms_default;             /* the same with the default shape            */
} psl_tuning;

/* reps >= 1 timed presolves per candidate (after one untimed). s: the settings
 * to tune (its thresholds and split are ignored); NULL = defaults. */
psl_status psl_tune(int32_t k, const psl_lp *lps, const psl_settings *s, int32_t reps, psl_tuning *out);

/* ---- Batched presolve -----------------------------------------------------
 * k independent LPs presolved together: they are laid out as the diagonal
 * blocks of one LP, so every kernel launch covers all of them, while each LP
 * keeps its own round count, stopping test and outer cycles. Each LP's
 * outcome, records and reduced problem are exactly those psl_presolve_run
 * gives for that LP alone, with the LP's own row and column numbering. */
typedef struct psl_batch psl_batch;

/* k >= 1 LPs, all with the same mem kind, each checked as at
 * psl_presolve_create (the message names the first invalid LP). The totals of
 * these LPs (rows, columns, nonzeros, and k) are the batch's capacity; their
 * total rows, columns and nnz must each be below 2^30. Settings apply to
 * every LP. */
psl_status psl_batch_create(int32_t k, const psl_lp *lps, const psl_settings *s, psl_batch **out);

/* Replace the LPs by k others (any shapes) whose totals fit the capacity,
 * reusing the device memory. PSL_ERR_CAPACITY otherwise. */
psl_status psl_batch_reload(psl_batch *b, int32_t k, const psl_lp *lps);

/* Presolve every LP. res[k] (host array of the batch's k) receives each
 * outcome; total (nullable) the batch's device times, rounds = the largest
 * round number of any LP, records / nnz / m_out / n_out summed over LPs. */
psl_status psl_batch_run(psl_batch *b, psl_result *res, psl_stats *total);

/* Statistics of LP idx of the last run: rounds, outer_cycles, records,
 * nnz_in, nnz_out, m_out, n_out (the times are the batch's). */
psl_status psl_batch_stats(const psl_batch *b, int32_t idx, psl_stats *out);

/* As psl_reduced_problem, for LP idx (device pointers into the batch's
 * arrays, valid until the next run, reload or free of the batch). */
psl_status psl_batch_reduced_problem(const psl_batch *b, int32_t idx, psl_reduced_view *out);

/* As psl_records, for LP idx (LP-local indices). */
psl_status psl_batch_records(const psl_batch *b, int32_t idx, int64_t *count, psl_record *out, int64_t cap);

/* As psl_postsolve, for LP idx (x, z have that LP's n entries, y its m). */
psl_status psl_batch_postsolve(psl_batch *b, int32_t idx, const double *x_red, const double *y_red,
                               const double *z_red, double *x, double *y, double *z);

void psl_batch_free(psl_batch *b);

/* Message of the last failure on b (or of the last failed batch create of
 * the thread when b is NULL). Never NULL. */
const char *psl_batch_last_error(const psl_batch *b);

/* ---- Serving ---------------------------------------------------------------
 * A request loop for a stream of LPs (continuous batching). Submitted LPs wait
 * in a FIFO queue; a free batch slot takes every waiting LP from the head of
 * the queue that fits its capacity and whose reduced problem can be reserved
 * in the device-memory budget, and presolves them as one batch. Several slots
 * run at once, each with its own stream, host thread and device arena, so LPs
 * that arrive while others are on the device start as soon as a slot and
 * memory are free and their work overlaps on the device. Reduced problems
 * stay on the device until released. Each request's outcome, records and
 * reduced problem are exactly those psl_presolve_run gives for its LP alone.
 * The server's functions may be called from any thread. */
typedef struct psl_server psl_server;

typedef struct {
    size_t hbm_budget_bytes;  /* device memory for the slot arenas and the
                                 resident reduced problems                   */
    int32_t slots;            /* batches in flight at once (>= 1)            */
    int32_t threaded;         /* 1: each slot has a worker thread; 0: no
                                 threads, the caller steps the server with
                                 psl_server_step                             */
    int32_t max_batch_lps;    /* LPs per batch                               */
    int32_t max_batch_rows, max_batch_cols;
    int64_t max_batch_nnz;    /* also the largest LP that can be served      */
    int32_t keep_original;    /* 1: a done ticket keeps its LP's rows and
                                 columns on the host (about 28 B per nonzero)
                                 so that psl_server_postsolve can undo
                                 FREE_SINGLETON records and give duals; 0
                                 (default): primal postsolve only, without
                                 FREE_SINGLETON records                      */
} psl_server_config;

/* Defaults: 64 GiB, 4 slots, threaded, 1024 LPs, 2.6e6 rows, 3.9e6 columns,
 * 3e7 nonzeros per batch. */
void psl_server_config_default(psl_server_config *c);

/* Create the slots (their arenas and streams) and the result heap (the rest
 * of the budget). settings.stream is ignored. PSL_ERR_CAPACITY if the arenas
 * do not fit the budget. */
psl_status psl_server_create(const psl_server_config *c, const psl_settings *s, psl_server **out);

/* Queue an LP; *ticket identifies the request. The LP's arrays (host or
 * device) are read when its batch starts: they must stay valid and unchanged
 * until the ticket is done. PSL_ERR_CAPACITY if the LP exceeds a batch or the
 * result heap; shape errors as at create (PSL_ERR_INVALID). */
psl_status psl_server_submit(psl_server *sv, const psl_lp *lp, uint64_t *ticket);

/* Without worker threads (threaded = 0): one step of the request loop. Every
 * free slot admits a batch of waiting LPs from the queue head (as a worker
 * would); every resident batch then advances by one unit of its run -- a
 * propagation round, an outer cycle's reduction pass, or the compaction --
 * with all slots' kernels queued before the step waits for any; batches
 * whose run ended are retired (their tickets done, reduced problems copied
 * to the result heap, records to the host). Nothing runs between steps.
 * *n_run = LPs resident during the step (0: the server is idle -- nothing
 * waiting, or the head does not fit yet). Steps called from several threads
 * run one after another. PSL_ERR_STATE if threaded. */
psl_status psl_server_step(psl_server *sv, int32_t *n_run);

/* Copy up to cap tickets completed since the last poll into tickets[], in
 * completion order; *n_done = how many. */
psl_status psl_server_poll(psl_server *sv, uint64_t *tickets, int32_t cap, int32_t *n_done);

/* Block until the ticket is done, or until timeout_ms (< 0: no limit) has
 * passed (then PSL_ERR_STATE). */
psl_status psl_server_wait(psl_server *sv, uint64_t ticket, double timeout_ms);

typedef struct {
    psl_status status;        /* PSL_OK, or why this request failed          */
    psl_result result;
    double queue_ms;          /* submit -> its batch started                 */
    double latency_ms;        /* submit -> reduced problem ready on device   */
    int32_t batch_lps;        /* LPs in its batch                            */
    int32_t slot;
    psl_stats stats;          /* as psl_batch_stats for this LP              */
} psl_ticket_info;

/* State of a done ticket (PSL_ERR_STATE while it is queued or running). */
psl_status psl_server_info(psl_server *sv, uint64_t ticket, psl_ticket_info *out);

/* The ticket's reduced problem, resident on the device until released. */
psl_status psl_server_reduced_problem(psl_server *sv, uint64_t ticket, psl_reduced_view *out);

/* The ticket's postsolve records (host copy; LP-local indices). */
psl_status psl_server_records(psl_server *sv, uint64_t ticket, int64_t *count, psl_record *out, int64_t cap);

/* As psl_postsolve, for the ticket's LP. A done ticket keeps its reduced
 * problem and records; the original matrix that the dual pass and the undoing
 * of FREE_SINGLETON records read is kept only when the server was created
 * with keep_original = 1. Without it, a non-NULL y_red, or a FREE_SINGLETON
 * record, gives PSL_ERR_UNSUPPORTED. */
psl_status psl_server_postsolve(psl_server *sv, uint64_t ticket, const double *x_red, const double *y_red,
                                const double *z_red, double *x, double *y, double *z);

/* Free the ticket's device memory and state. */
psl_status psl_server_release(psl_server *sv, uint64_t ticket);

/* Block until the queue is empty and no batch runs (without threads: step
 * the server until then; PSL_ERR_CAPACITY if the queue head cannot be
 * admitted on an idle server). */
psl_status psl_server_drain(psl_server *sv);

/* Device memory of the server: the slot arenas, the result heap's size, the
 * bytes reserved in it now and at most so far. A request reserves the size
 * of its LP's arrays (an upper bound of its reduced problem) at admission;
 * the reservation shrinks to the reduced problem when it is ready. */
psl_status psl_server_memory(psl_server *sv, size_t *arena_bytes, size_t *heap_bytes, size_t *heap_used,
                             size_t *heap_peak);

/* Stops the workers (waiting for running batches) and frees everything. */
void psl_server_free(psl_server *sv);

/* Message of the last failure on sv (or of the last failed server create of
 * the thread when sv is NULL). Never NULL. */
const char *psl_server_last_error(const psl_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* PSL_H */
