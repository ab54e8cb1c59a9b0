// psl_dev.h -- device state and device helpers of libpsl (gfx950, wave64).
//
// Layout in HBM (one presolver handle):
//   CSR   rp[m+1] i32, ci[N] i32, va[N] f64              (input, read-only)
//   CSC   cp[n+1] i32, ri[N] i32, cva[N] f64             (built at ingest)
//   rows  lhs/rhs[m] f64, row_on[m] u8, row_code[m] u8, row_out[m] 16 B
//   cols  bnd[n] double2 (lb, ub), bkey[2n] i64 (order-mapped accumulators of
//         the round's best lb / ub), src[2n] i32, col_len[n] i32, c[n] f64
//   bins  bins[m] {row, start, len} (active rows grouped by CSR length,
//         ascending within a bin; filtered as rows are removed)
// A column is removed exactly when lb == ub: a fixed column keeps lb = ub = v,
// and every active column has ub - lb > fix_tol * max(1, |lb|) >= 0 once a
// round has run, so the sweep learns a column's state from its bounds alone.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PSL_BLOCK 256
#define PSL_WAVE 64

namespace psl {

enum : uint8_t {
  REC_FIX_COL = 1, REC_EMPTY_COL = 2, REC_EMPTY_ROW = 3, REC_REDUNDANT_ROW = 4,
  REC_SINGLETON_ROW = 5, REC_BOUND_CHANGE = 6, REC_PARALLEL_ROW = 7, REC_LEADER_SIDES = 8,
  REC_DUAL_FIX = 9, REC_FREE_SINGLETON = 10, REC_PARALLEL_COL = 11, REC_LEADER_BOUNDS = 12,
  REC_FORCING_ROW = 13, REC_DOUBLETON_ROW = 14, REC_DOMINATED_COL = 15
};

// row decision codes written by the sweep for the current round
enum : uint8_t { RC_KEEP = 0, RC_EMPTY = 1, RC_REDUNDANT = 2, RC_SINGLETON = 3, RC_FORCE_MIN = 4, RC_FORCE_MAX = 5 };

// column decision bits of a round
enum : uint8_t {
  CC_LB = 1, CC_UB = 2, CC_FIX = 4, CC_EMPTY = 8, CC_UNBOUNDED = 16, CC_INFEAS = 32,
  CC_LBFIN = 64, CC_UBFIN = 128  // set at emission: lb (ub) went from infinite to finite
};
// a dual fixing sets both CC_FIX and CC_EMPTY (never set together otherwise)
#define CC_DUALFIX (CC_FIX | CC_EMPTY)

// row length bins: rows of <= 4 / <= 8 / <= 16 entries by 4- / 8- / 16-lane
// groups (the 8-lane bin is optional: its bound is 4 or 8), rows of <= 64 /
// <= 256 / <= 512 entries by one wavefront (1 / 4 / 8 contiguous positions per
// lane), longer rows split into workgroup chunks
enum { BIN_G4 = 0, BIN_G8 = 1, BIN_G16 = 2, BIN_W1 = 3, BIN_W4 = 4, BIN_W8 = 5, BIN_LONG = 6, NBINS = 7 };

#define PASS_LEN 2048      // positions per workgroup pass (256 lanes x 8)
#define LONG_MAX_CHUNKS 512
#define LONG_MAX_PASSES 64   // rows up to 512 chunks x 64 passes x 2048 positions

struct Record {
  uint8_t type, side;
  uint16_t round;
  int32_t i, j, k;
  double v[4];
};
static_assert(sizeof(Record) == 48, "record layout");

struct RowOut {      // what the sweep leaves for a removed row's record
  double v0, v1;     // (activity, -) / (min act, max act) / (a_ij, -)
  int32_t j, pad;
};

struct Cand {        // a candidate bound that may be the round's final value
  int32_t js;        // 2*j + side (side 1 = upper)
  int32_t pos;       // CSR position of the entry (its row and coefficient)
  double t;
};

struct LongChunk {   // one workgroup's slice of a long row: npass passes of PASS_LEN
  int32_t row, first;  // row index, first CSR position (relative to row start)
  int32_t lrow, npass; // index of the long row, passes per chunk
  int32_t cand_off;    // start of its candidate region (after the other bins')
  int32_t id;          // index of its partial statistics (stable under filtering)
};

struct BinEnt {      // one row of a bin list
  int32_t row, start, len, pad;
};

// Candidate regions: every sweep workgroup appends to its own region of the
// candidate buffer (an LDS counter, no global atomics). A region holds two
// candidates per position the workgroup can visit.

struct LongPart {    // partial statistics of one chunk (an aligned subtree)
  double smin, smax;
  int32_t nmin, nmax, L, tiny;  // tiny: active entries with |a| < coef_tol
};

struct LongRow {     // per long row
  int32_t row, chunk0, nchunk, npass;
};

// Batched presolve: K LPs form one block-diagonal LP (the rows and columns of
// LP k are contiguous, its entries use the shifted column indices). Every LP
// keeps its own round count and stopping state, so its records and reduced
// problem are those of presolving it alone.
struct LpFlags {     // per LP, cleared before every round
  int32_t infeasible, unbounded, merged, pad;
};

struct LpOut {       // per LP: nonzero when the last round gave it records (cleared per round)
  int32_t total, pad;
};

struct Flags {
  int32_t infeasible, unbounded, error, merged;
  int32_t cand_count, round_total, vlist_count, rows_removed;
  int32_t fin_cols;        // columns of the round with a bound that became finite
  int32_t mode;            // the next round's selection mode (bit 0: touched rows
                           // only, bit 1: inert rows skipped), set after a round
  int64_t error_pos;
  int32_t sel[NBINS + 4];  // the next round's selection: bin offsets [0..NBINS],
                           // rows, their nonzeros, long-row chunks
  int32_t lead_count;      // parallel pass: leaders whose merged sides add locks
  int32_t fs_total;        // free singleton eliminations of the round
  int32_t fs_rows;         // chunks of long eliminated rows listed
  int32_t fs_claims;       // chunks of long substituting rows listed
  int32_t dbl_count;       // doubleton-equality candidates listed
  int32_t dbl_applied;     // a doubleton substitution was applied this pass
};

struct Cfg {
  double feas_tol, fix_tol, min_improve, par_tol, inf_value, coef_tol;
  int32_t dual_fix;        // lock-based dual fixing on
  int32_t free_sing;       // zero-cost free column singletons eliminated
  int32_t forcing;         // forcing rows on
};

struct HashSlot {
  unsigned long long key;
  unsigned int leader;   // (inequality << 31) | row, minimised
  unsigned int pad;
};

struct Dev {
  int32_t m, n;
  int64_t nnz;
  const int32_t *rp, *ci;
  const double *va;
  const int32_t *cp, *ri;
  const double *cva;
  double *lhs, *rhs;
  double2 *bnd;
  long long *bkey;
  int32_t *src;
  double *c;                   // costs (a working copy: substitutions change them)
  unsigned long long *owner;   // free singletons: per column the lowest claim, (~round << 32) | row,
                               // so a claim of the current round beats an older one (reset per run)
  uint8_t *fs_bad;             // per row: a long substituting row lost a column
  int32_t *col_len;
  uint8_t *row_on, *row_code, *col_code;
  uint8_t *dirty;          // rows touched by a column change since last swept
  uint8_t *dirty_tile;     // per 1024 rows: some row of it was marked (the row
                           // selection skips the other tiles when it takes
                           // marked rows only)
  const int32_t *rowid1;   // row of CSR position p at index p + 1 (built at ingest)
  int2 *rinf;              // per row: infinite min / max contributions at its last
                           // sweep, lowered as bounds of its columns become finite
  int32_t *dense_cols;     // columns of more than 4096 entries (listed at ingest)
  int32_t *n_dense;
  uint8_t *touch;          // columns whose decision may change this round
  unsigned long long *locks;  // dual fixing: per column, the alive rows keeping it
                              // from decreasing (low 32 bits) / increasing (high)
  // free singletons: per column and side, -1 = infinite input bound not changed,
  // r >= 0 = infinite input bound tightened only from row r, -2 = otherwise
  int32_t *lsrc, *usrc;
  uint8_t *fs_flag;        // column to check for a free singleton this round
  int32_t *fs_pick;        // per row: lowest candidate column (INT32_MAX: none)
  const uint32_t *colid;   // column of each position of the transposed copy
  RowOut *row_out;
  Cand *cand;
  int32_t *cand_cnt;   // candidates written per sweep workgroup
  Flags *flags;
  int32_t *cnt, *off;
  Record *rec;
  const BinEnt *bins;
  int32_t bin_off[NBINS + 1];
  const LongChunk *lchunk;
  const LongChunk *chunks0;    // chunk table of all long rows (built at ingest)
  LongPart *lpart;
  LongRow *lrow;
  int32_t nlong, nchunks;
  // batched presolve (K LPs); with K == 1 every row and column is in LP 0
  // and none of these arrays is read
  int32_t K;
  const int32_t *row_lp, *col_lp;     // LP of each row / column
  const int32_t *lp_row0, *lp_col0;   // [K+1] first row / column of each LP
  uint8_t *lp_ok;                     // [K] LP still presolving (its rows stay in the bins;
                                      // cleared here when the LP stops)
  const int32_t *lp_round;            // [K] the LP's own number of the current round
  LpFlags *lpf;                       // [K]
  LpOut *lpo;                         // [K]
  Cfg cfg;
};

__device__ __forceinline__ int row_lp_of(const Dev& d, int i) { return d.K > 1 ? d.row_lp[i] : 0; }
__device__ __forceinline__ int col_lp_of(const Dev& d, int j) { return d.K > 1 ? d.col_lp[j] : 0; }
// round number written into a record of LP lp
__device__ __forceinline__ int round_of(const Dev& d, int lp, int round) { return d.K > 1 ? d.lp_round[lp] : round; }
// an LP that stops leaves the next selection at once
__device__ __forceinline__ void flag_infeasible(const Dev& d, int lp) {
  atomicOr(&d.flags->infeasible, 1);
  if (d.K > 1) {
    atomicOr(&d.lpf[lp].infeasible, 1);
    d.lp_ok[lp] = 0;
  }
}
__device__ __forceinline__ void flag_unbounded(const Dev& d, int lp) {
  atomicOr(&d.flags->unbounded, 1);
  if (d.K > 1) {
    atomicOr(&d.lpf[lp].unbounded, 1);
    d.lp_ok[lp] = 0;
  }
}

// ---------------------------------------------------------------------------
// scalar helpers (IEEE double; the library is built with -ffp-contract=off)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double pos0(double x) { return x == 0.0 ? 0.0 : x; }
__device__ __forceinline__ double mx1(double x) {
  double a = fabs(x);
  return a > 1.0 ? a : 1.0;
}
__device__ __forceinline__ bool is_inf(double x) { return __builtin_isinf(x); }

// the locks one row puts on a column with coefficient a (down in the low
// word, up in the high word): a > 0 with a finite lhs (a < 0: rhs) keeps the
// column from decreasing, a > 0 with a finite rhs (a < 0: lhs) from increasing
__device__ __forceinline__ unsigned long long lock_bits(double a, double lhs, double rhs) {
  unsigned long long lf = is_inf(lhs) ? 0ull : 1ull, rf = is_inf(rhs) ? 0ull : 1ull;
  return a > 0 ? (lf | (rf << 32)) : (rf | (lf << 32));
}

// a row removal takes column j (coefficient a, the row's sides lhs / rhs) out
// of that row; a column left in no row is decided this round, and with dual
// fixing so is every column that lost a row (it may have lost its last lock);
// a column left in one row is checked for a free singleton
__device__ __forceinline__ void drop_col(const Dev& d, int j, double a, double lhs, double rhs) {
  int left = atomicSub(&d.col_len[j], 1) - 1;
  if (d.cfg.dual_fix) {
    atomicAdd(&d.locks[j], 0ull - lock_bits(a, lhs, rhs));  // the counts never go below 0
    d.touch[j] = 1;
  } else if (left == 0) {
    d.touch[j] = 1;
  }
  if (d.cfg.free_sing && left == 1) d.fs_flag[j] = 1;  // now in one row: a candidate
}

// A row whose every finite side has at least two infinite contributions on
// the side's residual, and that cannot be redundant, gives no candidate, no
// removal and no infeasibility: sweeping it changes nothing.
__device__ __forceinline__ bool row_inert(int2 c, double lhs, double rhs) {
  bool lo_inf = is_inf(lhs), up_inf = is_inf(rhs);
  bool prop = (!up_inf && c.x <= 1) || (!lo_inf && c.y <= 1);
  bool redundant_possible = (lo_inf || c.x == 0) && (up_inf || c.y == 0);
  return !prop && !redundant_possible;
}

__device__ __forceinline__ double tol_of(const Cfg& c, double x) { return c.feas_tol * mx1(x); }

// order-preserving map double <-> int64 (an involution); -0 never occurs
__device__ __forceinline__ long long dkey(double x) {
  long long b = __double_as_longlong(x);
  return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFLL);
}
__device__ __forceinline__ double dunkey(long long k) {
  return __longlong_as_double(k >= 0 ? k : (k ^ 0x7FFFFFFFFFFFFFFFLL));
}

// contribution of coefficient a on [lb, ub] to the min / max activity
__device__ __forceinline__ void contrib(double a, double lb, double ub, double& tmin,
                                       bool& imin, double& tmax, bool& imax) {
  double bmin = a > 0 ? lb : ub;
  double bmax = a > 0 ? ub : lb;
  imin = is_inf(bmin);
  imax = is_inf(bmax);
  tmin = imin ? 0.0 : pos0(a * bmin);
  tmax = imax ? 0.0 : pos0(a * bmax);
}

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & (PSL_WAVE - 1); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ double shfl_xor_d(double x, int m) {
  return __shfl_xor(x, m, PSL_WAVE);
}

// Sum over aligned groups of G lanes by a butterfly. fl(a + b) is
// commutative, so both partners compute the same node and after log2(G)
// steps every lane of the group holds the pairwise tree over its G lanes.
template <int G>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
  for (int s = 1; s < G; s <<= 1) x = x + shfl_xor_d(x, s);
  return x;
}

template <int G>
__device__ __forceinline__ unsigned long long group_sum_u64(unsigned long long x) {
#pragma unroll
  for (int s = 1; s < G; s <<= 1) {
    unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
    lo = __shfl_xor(lo, s, PSL_WAVE);
    hi = __shfl_xor(hi, s, PSL_WAVE);
    x += ((unsigned long long)hi << 32) | lo;
  }
  return x;
}

template <int G>
__device__ __forceinline__ unsigned long long group_mask() {
  if constexpr (G == 64) return ~0ull;
  else return ((1ull << G) - 1) << (lane_id() & ~(G - 1));
}

// Pairwise tree over v[0..n) padded with +0 to the next power of two,
// in place (used for pass and chunk sums held in LDS).
__device__ __forceinline__ double tree_inplace(double* v, int n) {
  if (n <= 0) return 0.0;
  int p = 1;
  while (p < n) p <<= 1;
  for (int w = 1; w < p; w <<= 1)
    for (int i = 0; i + w < n; i += 2 * w) v[i] = v[i] + v[i + w];
  return v[0];
}

// Wave-aggregated append of one 16-byte candidate per lane with pred set;
// counter may live in LDS. Must be reached by all lanes of the wave.
__device__ __forceinline__ void wave_append(bool pred, const Cand& e, Cand* list, int32_t* counter) {
  unsigned long long mask = __ballot(pred);
  if (mask == 0) return;
  int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (int)__popcll(mask));
  base = __shfl(base, leader, PSL_WAVE);
  if (pred) list[base + __popcll(mask & lanemask_lt())] = e;
}

// candidate-region sizes (entries) of the sweep bins, per workgroup
// Row blocks (of 256 threads' rows) one workgroup of a bin sweeps in turn:
// short rows give a wavefront little work, so their workgroups take several.
__host__ __device__ __forceinline__ int bin_rep(int bin) {
  return bin <= BIN_G16 ? 4 : bin == BIN_W1 ? 2 : 1;
}

// rows of a row block of the bin
__host__ __device__ __forceinline__ int bin_rows(int bin) {
  return bin == BIN_G4 ? 64 : bin == BIN_G8 ? 32 : bin == BIN_G16 ? 16 : 4;
}

__host__ __device__ __forceinline__ int64_t cand_region(int bin) {
  // 2 candidates x (rows per workgroup x longest row of the bin)
  int len = bin == BIN_G4 ? 4 : bin == BIN_G8 ? 8 : bin == BIN_G16 ? 16 : bin == BIN_W1 ? 64 : bin == BIN_W4 ? 256 : 512;
  return 2 * (int64_t)bin_rep(bin) * bin_rows(bin) * len;
}

// SplitMix64 output function for state x (Steele, Lea & Flood 2014).
__device__ __forceinline__ unsigned long long splitmix(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// sign, exponent and top 32 mantissa bits, rounded to nearest
__device__ __forceinline__ unsigned long long quantize(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  unsigned long long sign = b >> 63;
  unsigned long long mag = b & 0x7FFFFFFFFFFFFFFFULL;
  return ((mag + (1ULL << 19)) >> 20) | (sign << 63);
}

// exclusive scan of one int per thread across a block of NT threads
template <int NT>
__device__ __forceinline__ int block_excl_scan_n(int v, int* total) {
  __shared__ int wsum[NT / PSL_WAVE];
  int lane = lane_id(), w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < PSL_WAVE; o <<= 1) {
    int y = __shfl_up(x, o, PSL_WAVE);
    if (lane >= o) x += y;
  }
  if (lane == PSL_WAVE - 1) wsum[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / PSL_WAVE; ++k) {
    int s = wsum[k];
    if (k < w) pre += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

// the same across the 256-thread block
__device__ __forceinline__ int block_excl_scan(int v, int* total) { return block_excl_scan_n<PSL_BLOCK>(v, total); }


}  // namespace psl
