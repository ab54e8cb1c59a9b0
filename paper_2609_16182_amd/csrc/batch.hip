// batch.hip -- batched presolve: K independent LPs presolved as the blocks
// of one block-diagonal LP.
//
// The LPs keep their own numbering where a result depends on it (the
// parallel-row keys hash LP-local column indices, records and reduced
// problems are renumbered per LP), and their own round counts and stopping
// state (kept on the host), so every LP gets the result of presolving it
// alone. These kernels load the union, map rows and columns to their LPs,
// and split the record stream by LP.
#include <utility>

#include "psl_kern.h"
#include "sweep.h"

namespace psl {

// last k in [lo, hi] with start[k] <= x (start ascending, start[lo] <= x)
template <class T>
__device__ __forceinline__ int find_seg(const T* start, int lo, int hi, int64_t x) {
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((int64_t)start[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// LP range of the block's elements [b0, b1) (b1 > b0), in LDS
template <class T>
__device__ __forceinline__ void block_seg_range(const T* start, int K, int64_t b0, int64_t b1, int& lo, int& hi) {
  __shared__ int r[2];
  if (threadIdx.x == 0) {
    r[0] = find_seg(start, 0, K - 1, b0);
    r[1] = find_seg(start, r[0], K - 1, b1 - 1);
  }
  __syncthreads();
  lo = r[0];
  hi = r[1];
}

#define BG_ITEMS 8
#define BG_TILE (PSL_BLOCK * BG_ITEMS)

__device__ __forceinline__ void report_err(const Dev& d, int32_t bit, int64_t pos) {
  atomicOr(&d.flags->error, bit);
  atomicMin((long long*)&d.flags->error_pos, (long long)pos);
}

// rows: row pointers shifted by the LP's first position, sides, row -> LP
__global__ void __launch_bounds__(PSL_BLOCK) k_bg_rows(Dev d, const LpDesc* desc, const int64_t* z0, int32_t* rp,
                                                       double* lhs, double* rhs, int32_t* row_lp) {
  int64_t b0 = (int64_t)blockIdx.x * BG_TILE, b1 = b0 + BG_TILE;
  if (b1 > d.m) b1 = d.m;
  if (b0 >= b1) return;
  int lo, hi;
  block_seg_range(d.lp_row0, d.K, b0, b1, lo, hi);
  for (int64_t i = b0 + threadIdx.x; i < b1; i += PSL_BLOCK) {
    int k = find_seg(d.lp_row0, lo, hi, i);
    LpDesc L = desc[k];
    int q = (int)(i - d.lp_row0[k]);
    int a = L.rp[q];
    if ((q == 0 && a != 0) || (q == L.m - 1 && (int64_t)L.rp[q + 1] != L.nnz)) report_err(d, 1, i);
    rp[i] = (int32_t)(a + z0[k]);
    lhs[i] = L.lhs[q];
    rhs[i] = L.rhs[q];
    row_lp[i] = k;
  }
}

__global__ void __launch_bounds__(PSL_BLOCK) k_bg_cols(Dev d, const LpDesc* desc, double* lb, double* ub, double* c,
                                                       int32_t* col_lp) {
  int64_t b0 = (int64_t)blockIdx.x * BG_TILE, b1 = b0 + BG_TILE;
  if (b1 > d.n) b1 = d.n;
  if (b0 >= b1) return;
  int lo, hi;
  block_seg_range(d.lp_col0, d.K, b0, b1, lo, hi);
  for (int64_t j = b0 + threadIdx.x; j < b1; j += PSL_BLOCK) {
    int k = find_seg(d.lp_col0, lo, hi, j);
    LpDesc L = desc[k];
    int q = (int)(j - d.lp_col0[k]);
    lb[j] = L.lb[q];
    ub[j] = L.ub[q];
    c[j] = L.c[q];
    col_lp[j] = k;
  }
}

// entries: column indices checked against the LP's own column count, then shifted
__global__ void __launch_bounds__(PSL_BLOCK) k_bg_entries(Dev d, const LpDesc* desc, const int64_t* z0, int32_t* ci,
                                                          double* va) {
  int64_t b0 = (int64_t)blockIdx.x * BG_TILE, b1 = b0 + BG_TILE;
  if (b1 > d.nnz) b1 = d.nnz;
  if (b0 >= b1) return;
  int lo, hi;
  block_seg_range(z0, d.K, b0, b1, lo, hi);
  for (int64_t p = b0 + threadIdx.x; p < b1; p += PSL_BLOCK) {
    int k = find_seg(z0, lo, hi, p);
    const LpDesc& L = desc[k];
    int64_t q = p - z0[k];
    int j = L.ci[q];
    if (j < 0 || j >= L.n) {
      report_err(d, 2, p);
      j = 0;
    }
    ci[p] = j + d.lp_col0[k];
    va[p] = L.va[q];
  }
}

// row -> LP and column -> LP maps (host-loaded batches)
__global__ void __launch_bounds__(PSL_BLOCK) k_lp_maps(Dev d, int32_t* row_lp, int32_t* col_lp) {
  int64_t t = (int64_t)blockIdx.x * BG_TILE;
  int64_t span = (int64_t)d.m + d.n;
  int64_t b1 = t + BG_TILE < span ? t + BG_TILE : span;
  for (int64_t x = t + threadIdx.x; x < b1; x += PSL_BLOCK) {
    if (x < d.m) row_lp[x] = find_seg(d.lp_row0, 0, d.K - 1, x);
    else col_lp[x - d.m] = find_seg(d.lp_col0, 0, d.K - 1, x - d.m);
  }
}

// LP of each record: its row for row records, its column for column records
__global__ void k_rec_keys(Dev d, const Record* rec, int64_t count, uint32_t* keys) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  Record r = rec[t];
  bool col = r.type == REC_FIX_COL || r.type == REC_EMPTY_COL || r.type == REC_BOUND_CHANGE ||
             r.type == REC_DUAL_FIX || r.type == REC_PARALLEL_COL || r.type == REC_LEADER_BOUNDS ||
             r.type == REC_DOMINATED_COL;
  keys[t] = (uint32_t)(col ? d.col_lp[r.j] : d.row_lp[r.i]);
}

__device__ __forceinline__ int32_t local_idx(int32_t v, int32_t base) {
  return v >= 0 && v != 0x7FFFFFFF ? v - base : v;
}

// records in LP order (stable), renumbered to LP-local rows and columns;
// rec_off[k] = first record of LP k, rec_off[K] = count
__global__ void k_rec_gather(Dev d, const Record* rec, const uint32_t* keys, const int32_t* idx, int64_t count,
                             Record* out, int32_t* rec_off) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int k = (int)keys[t];
  Record r = rec[idx[t]];
  int i0 = d.lp_row0[k], j0 = d.lp_col0[k];
  switch (r.type) {
    case REC_FIX_COL:
    case REC_EMPTY_COL:
    case REC_DUAL_FIX:
    case REC_DOMINATED_COL:
    case REC_LEADER_BOUNDS:
      r.j = local_idx(r.j, j0);
      break;
    case REC_PARALLEL_COL:
      r.j = local_idx(r.j, j0);
      r.k = local_idx(r.k, j0);
      break;
    case REC_BOUND_CHANGE:
      r.j = local_idx(r.j, j0);
      r.k = local_idx(r.k, i0);
      break;
    case REC_SINGLETON_ROW:
    case REC_FREE_SINGLETON:
      r.i = local_idx(r.i, i0);
      r.j = local_idx(r.j, j0);
      break;
    case REC_PARALLEL_ROW:
      r.i = local_idx(r.i, i0);
      r.k = local_idx(r.k, i0);
      break;
    case REC_LEADER_SIDES:
      r.i = local_idx(r.i, i0);
      r.j = local_idx(r.j, i0);
      r.k = local_idx(r.k, i0);
      break;
    case REC_DOUBLETON_ROW:
      r.i = local_idx(r.i, i0);
      r.j = local_idx(r.j, j0);
      r.k = local_idx(r.k, j0);
      break;
    default:
      r.i = local_idx(r.i, i0);
      break;
  }
  out[t] = r;
  int prev = t == 0 ? -1 : (int)keys[t - 1];
  for (int q = prev + 1; q <= k; ++q) rec_off[q] = (int32_t)t;
  if (t == count - 1)
    for (int q = k + 1; q <= d.K; ++q) rec_off[q] = (int32_t)count;
}

// ---------------------------------------------------------------------------
static unsigned tiles(int64_t n) { return (unsigned)((n + BG_TILE - 1) / BG_TILE); }

void batch_gather(const Dev& d, const LpDesc* desc, const int64_t* z0, int32_t* rp, int32_t* ci, double* va,
                  double* lhs, double* rhs, double* lb, double* ub, double* c, int32_t* row_lp, int32_t* col_lp,
                  hipStream_t s) {
  if (d.m > 0) hipLaunchKernelGGL(k_bg_rows, dim3(tiles(d.m)), dim3(PSL_BLOCK), 0, s, d, desc, z0, rp, lhs, rhs, row_lp);
  if (d.n > 0) hipLaunchKernelGGL(k_bg_cols, dim3(tiles(d.n)), dim3(PSL_BLOCK), 0, s, d, desc, lb, ub, c, col_lp);
  if (d.nnz > 0) hipLaunchKernelGGL(k_bg_entries, dim3(tiles(d.nnz)), dim3(PSL_BLOCK), 0, s, d, desc, z0, ci, va);
}

void batch_maps(const Dev& d, int32_t* row_lp, int32_t* col_lp, hipStream_t s) {
  int64_t span = (int64_t)d.m + d.n;
  if (span > 0) hipLaunchKernelGGL(k_lp_maps, dim3(tiles(span)), dim3(PSL_BLOCK), 0, s, d, row_lp, col_lp);
}

size_t rec_split_ws_ints(int64_t count) { return radix_ws_ints(count); }

void rec_split(const Dev& d, const Record* rec, int64_t count, Record* out, int32_t* rec_off, uint32_t* k0,
               uint32_t* k1, int32_t* v0, int32_t* v1, int32_t* ws, hipStream_t s) {
  // K > 1 here, so at least one radix pass runs and v0 ends as the permutation
  if (count == 0) {
    fill_i32(rec_off, 0, d.K + 1, s);
    return;
  }
  unsigned blocks = (unsigned)((count + PSL_BLOCK - 1) / PSL_BLOCK);
  hipLaunchKernelGGL(k_rec_keys, dim3(blocks), dim3(PSL_BLOCK), 0, s, d, rec, count, k0);
  int bits = 0;
  while ((1 << bits) < d.K) ++bits;
  const int32_t* vin = nullptr;
  for (int sh = 0; sh < bits; sh += 8) {
    int b = bits - sh < 8 ? bits - sh : 8;
    radix_pass(k0, vin, k1, v1, count, sh, b, ws, s);
    std::swap(k0, k1);
    std::swap(v0, v1);
    vin = v0;
  }
  hipLaunchKernelGGL(k_rec_gather, dim3(blocks), dim3(PSL_BLOCK), 0, s, d, rec, (const uint32_t*)k0,
                     (const int32_t*)v0, count, out, rec_off);
}

}  // namespace psl
