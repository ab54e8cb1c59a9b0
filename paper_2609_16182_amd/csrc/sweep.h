// sweep.h -- launchers of the per-round kernels (sweep.hip), the parallel-row
// pass (parallel.hip), ingest (ingest.hip) and compaction (compact.hip).
#pragma once
#include "bits.h"
#include "psl_dev.h"

namespace psl {

enum { MODE_ROUND = 0, MODE_COMPACT = 1 };

struct SweepGrid {
  int nb[NBINS];        // workgroups per bin in the fused sweep launch
  int64_t long_base;    // candidate entries before the long-row regions
};

// candidate region start of sweep workgroup b (non-long bins)
__host__ __device__ __forceinline__ int64_t cand_region_start(const SweepGrid& g, int b, int& bin) {
  int64_t off = 0;
  for (bin = 0; bin < BIN_LONG; ++bin) {
    if (b < g.nb[bin]) return off + (int64_t)b * cand_region(bin);
    b -= g.nb[bin];
    off += (int64_t)g.nb[bin] * cand_region(bin);
  }
  return -1;  // a long-row chunk: region from its chunk record
}

// sweep.hip
void launch_long_stats(const Dev& d, int mode, hipStream_t s);
void launch_sweep(const Dev& d, const SweepGrid& g, int mode, hipStream_t s);
void launch_long_consts(const Dev& d, hipStream_t s);
void launch_src(const Dev& d, const SweepGrid& g, hipStream_t s);
// decisions, counts and records of a round (tile_sum / tile_off: one int per
// 1024 rows and columns, ws: scan workspace)
void launch_decide(const Dev& d, int64_t base, int round, int32_t* tile_sum, int32_t* tile_off, int32_t* ws,
                   hipStream_t s);
int long_max_passes();

// ingest.hip
struct IngestScratch {
  int32_t* rowid1;   // [nnz+1]: rowid1[p+1] = row of CSR position p
  uint32_t* k0;      // [nnz]
  uint32_t* k1;      // [nnz]
  int32_t* v0;       // [nnz]
  int32_t* v1;       // [nnz]
  int32_t* ws;       // scan / radix workspace
};
void launch_check_rows(const Dev& d, hipStream_t s);
void check_cols(const Dev& d, const double* lb_in, const double* ub_in, double* c_mut, hipStream_t s);
void launch_check_entries(const Dev& d, const int32_t* rowid1, hipStream_t s);
void build_rowid(const Dev& d, IngestScratch& sc, hipStream_t s);
// transposed copy (vtmp: nnz doubles of scratch); returns the column of each
// of its positions
const uint32_t* build_csc(const Dev& d, int32_t* cp, int32_t* ri, double* cva, int32_t* col_len, IngestScratch& sc,
                          double* vtmp, hipStream_t s);
// bins: writes the bin lists and per-bin counts (device counts[NBINS])
void build_bins(const Dev& d, const int32_t* thresholds, BinEnt* bins, int32_t* counts, IngestScratch& sc,
                hipStream_t s);
// The rows a round sweeps: every active row of an LP still presolving (and,
// by the mode, only the marked ones / none that is inert) as bin lists in row
// order in out, the kept long rows' chunks (from d.chunks0) in cout, and
// sel = {bin offsets [0..NBINS], rows, nonzeros, chunks} (device). The mode
// is *mode_dev (device: bit 0 marked rows only, bit 1 inert rows skipped), or
// mode_host when mode_dev is null. Kept rows' marks are cleared. keep:
// select_keep_bytes(m) bytes, cnt: select_count_ints(m) ints.
size_t select_keep_bytes(int64_t m);
size_t select_count_ints(int64_t m);
void select_rows(const Dev& d, const int32_t* mode_dev, int mode_host, int t_long, int t_g8, uint8_t* keep,
                 int32_t* cnt, BinEnt* out, LongChunk* cout, int32_t* sel, int32_t* ws, hipStream_t s);
// after a round: decide on the device the next round's mode (d.flags->mode:
// bit 0 = sweep the touched rows only, allowed with allow_incremental when
// fewer than n / incr_factor columns changed; bit 1 = keep the infinite-
// contribution counts, when fewer than n / count_factor bounds became
// finite); with bit 1, lower the counts of the rows of columns whose bounds
// became finite; with bit 0, mark the rows of the changed columns dirty
void mark_dirty(const Dev& d, bool allow_incremental, int incr_factor, int count_factor, hipStream_t s);
// d.dense_cols / d.n_dense from the transposed copy (after build_csc)
void list_dense_cols(const Dev& d, hipStream_t s);
// chunk table of the long rows (d.nlong set); total chunks to *total (device)
// totals[0] = chunks, totals[1] = candidate units of all chunks
void build_long_chunks(const Dev& d, int npass0, LongChunk* chunks, int32_t* cnt, int32_t* cnt2, int32_t* totals,
                       int32_t* ws, hipStream_t s);
void launch_round0_count(const Dev& d, hipStream_t s);
void launch_round0_emit(const Dev& d, int64_t base, hipStream_t s);
void launch_init_state(const Dev& d, hipStream_t s);
// d.locks of every column from the alive rows (dual fixing); dn, up: nnz + 1
// ints of scratch each, ws: scan workspace for nnz + 1 items
void init_locks(const Dev& d, int32_t* dn, int32_t* up, int32_t* ws, hipStream_t s);

// parcols.hip: parallel columns, after the parallel-row pass (records from
// base + d.flags->round_total, which it raises by its own count; merged LPs
// flagged in d.flags->merged / d.lpf). Scratch of n entries each:
struct ColScratch {
  uint64_t* key;            // per column: its 63-bit key (all ones: no candidate)
  uint32_t *keys, *keys2;   // sort keys (the key's low, then high half)
  int32_t *vals, *vals2;    // sort payload (columns)
  int32_t* lead;            // per column: its leader (itself for a leader), else -1
  double* lam;              // per merged column: lambda
  double2* nb;              // per leader: merged interval
  double2* terms;           // per sorted position: a merged member's scaled interval
  int32_t* total;           // [1] records
};
size_t par_cols_ws_ints(int64_t n);
void launch_par_cols(const Dev& d, const ColScratch& P, int64_t base, int round, int32_t* ws, hipStream_t s);

// singleton.hip: zero-cost free column singletons at the end of a round
// (records from base + the round's record total; list: nnz / 32 + m ints of
// scratch; adds its records to d.flags->round_total and its rows to
// rows_removed)
void launch_free_singletons(const Dev& d, int32_t* list, int64_t base, int round, int32_t* ws, hipStream_t s);

// parallel.hip
struct LpTab {        // an LP's slice of the parallel-row table
  int64_t base, cap;  // first slot, slots (a power of two)
};
struct ParScratch {
  HashSlot* table;
  int64_t cap;        // power of two (all slots when K > 1)
  const LpTab* lpt;   // [K] per-LP slices (K > 1)
  int32_t* slot;      // [m] slot of a candidate row, -1 otherwise
  int32_t* lead;      // [m] leader of a merged row, -1 otherwise
  long long* side_key;// [2m] merged (lhs, rhs) keys of a leader
  int32_t* side_src;  // [2m]
  uint8_t* is_leader; // [m]
  int32_t* vlist;     // [m] rows to verify
  unsigned long long* hacc;  // [4 * long rows] hash accumulators (h1, h2, L)
                             // and the row's first active coefficient (bits)
  double* lam;        // [m] lambda of a verified row (a_r = lambda a_leader)
  uint64_t* abits;    // [n/64+1] active columns (lb != ub), one bit each
};
void launch_par_reset(const Dev& d, const ParScratch& p, hipStream_t s);
void launch_par_hash(const Dev& d, const ParScratch& p, const SweepGrid& g, hipStream_t s);
void launch_par_verify(const Dev& d, const ParScratch& p, hipStream_t s);
void launch_par_count(const Dev& d, const ParScratch& p, hipStream_t s);
void launch_par_emit(const Dev& d, const ParScratch& p, int64_t base, int round, hipStream_t s);
void launch_par_drop(const Dev& d, const ParScratch& p, hipStream_t s);

// doubleton.hip: doubleton-equality substitution (allocated when enabled)
// a rewrite of a long row that inserts the kept column (entries move by one
// over up to the whole row), done by a workgroup after the substitutions
struct DblTask {
  int32_t r, k, j, pad;  // row, eliminated column, kept column
  double v;              // the kept column's new coefficient
};
struct DblScratch {
  int32_t* list;       // [m] candidate rows
  int32_t *cj, *ck;    // [m] kept / eliminated column of a candidate (-1: none)
  double *aj, *ak, *b; // [m] its coefficients and right-hand side
  int32_t* row_claim;  // [m] lowest claiming candidate of each row
  int32_t* col_claim;  // [n] ... of each column
  uint8_t* col_mod;    // [n] kept by an earlier substitution (for the run)
  int32_t* by;         // [n] applied row whose kept column this is, -1
  double2* tb;         // [n] interval x_k's bounds give a kept column
  int32_t* total;      // [2] records: rows, transferred bounds
  DblTask* long_task;  // [doubleton_long_cap(nnz)] deferred long-row rewrites
  int32_t* long_cnt;   // [1]
};
int64_t doubleton_long_cap(int64_t nnz);  // rows longer than the lane-rewrite limit, at most
void launch_doubletons(const Dev& d, const DblScratch& S, int64_t base, int round, int32_t* ws, hipStream_t s);
void launch_doubleton_relock(const Dev& d, const DblScratch& S, hipStream_t s);
void launch_doubleton_init(const Dev& d, const DblScratch& S, hipStream_t s);  // no column kept yet

// dominated.hip: dominated columns through implied dual bounds (allocated
// when enabled); records from base + the pass's record total, added to it
struct DomScratch {
  long long* ykey;     // [2m] order-mapped bounds (lower, upper) of each row's dual
  int8_t* side;        // [n] the fixing of each column: 0 lower, 1 upper, -1 none
  int32_t* lp_flag;    // [K] crossing dual bounds: 1 skip the LP, 2 unbounded
  int32_t* total;      // [1] records
};
void launch_dominated(const Dev& d, const DomScratch& S, int64_t base, int round, int32_t* ws, hipStream_t s);

// compact.hip
struct Reduced {
  int32_t *row_ptr, *col_idx, *col_ptr, *row_idx, *row_map, *col_map;
  double *val, *cval, *lhs, *rhs, *lb, *ub, *c;
  uint8_t *row_class, *col_class;
};
struct LpRed {           // bases of an LP's reduced problem in the batch's arrays
  int32_t rb, cb;        // first reduced row / column
  int32_t eb, qb;        // first position in the reduced CSR / transposed copy
};
struct CompactScratch {
  int32_t* row_new;       // [m]     kept flags -> new row ids
  int32_t* col_new;       // [n]     kept flags -> new column ids
  uint8_t* col_keep;      // [n]     kept columns (bytes)
  RankWord* rbits;        // [m/64+1] kept rows, one bit each, with ranks
  RankWord* cbits;        // [n/64+1] kept columns, one bit each, with ranks
  double* terms;          // [n]     cost terms of removed columns
  double* pws;            // pairwise-sum workspace; pws[0] = the sum
  int32_t* totals;        // [4]     m', n', nnz' (CSR), nnz' (transposed)
  double* offset;         // [1]     reduced objective offset
  int32_t* ws;            // scan workspace
  int32_t* eflag;         // [nnz+1] CSR keep flags -> output positions
  int32_t* qflag;         // [nnz+1] transposed keep flags -> output positions
  const int32_t* rowid1;  // row of CSR position p at index p + 1
  const uint32_t* colid;  // column of each position of the transposed copy
  LpRed* lpr;             // [K+1] per-LP bases (lpr[K] = totals)
  const int32_t* seg;     // [K+1] first column of each LP (K > 1), device
  const int32_t* seg_host;//        the same on the host
  const double* lp_off_in;// [K] input objective offsets (K > 1)
};
// flags and scans (totals written to c.totals)
void compact_flags(const Dev& d, const CompactScratch& c, hipStream_t s);
// offset(s), gather of both layouts, vectors, maps and classes; with K > 1 the
// offsets go to c.offset[0..K)
void compact_write(const Dev& d, const CompactScratch& c, const Reduced& r, double obj_offset, hipStream_t s);

// batch.hip
struct LpDesc {        // one LP of a batch, as given (device pointers)
  const int32_t *rp, *ci;
  const double *va, *lhs, *rhs, *lb, *ub, *c;
  int32_t m, n;
  int64_t nnz;
};
// union arrays from K device-resident LPs (d.m, d.n, d.nnz, d.K, d.lp_row0,
// d.lp_col0 set; z0[k] = first position of LP k); errors go to d.flags
void batch_gather(const Dev& d, const LpDesc* desc, const int64_t* z0, int32_t* rp, int32_t* ci, double* va,
                  double* lhs, double* rhs, double* lb, double* ub, double* c, int32_t* row_lp, int32_t* col_lp,
                  hipStream_t s);
// row -> LP and column -> LP maps from d.lp_row0 / d.lp_col0
void batch_maps(const Dev& d, int32_t* row_lp, int32_t* col_lp, hipStream_t s);
// stable split of the records by LP, renumbered per LP (K > 1); scratch of
// count entries each, ws: rec_split_ws_ints(count)
size_t rec_split_ws_ints(int64_t count);
void rec_split(const Dev& d, const Record* rec, int64_t count, Record* out, int32_t* rec_off, uint32_t* k0,
               uint32_t* k1, int32_t* v0, int32_t* v1, int32_t* ws, hipStream_t s);

}  // namespace psl
