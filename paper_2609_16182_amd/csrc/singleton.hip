// singleton.hip -- elimination of zero-cost free column singletons (section
// 3.2, "Column singletons"): a column with c_j = 0 in one alive row i, whose
// bounds are infinite or were tightened only from row i (so they are implied
// by it), can take any value row i needs; row i and the column leave
// together and postsolve recovers x_j from the row. With c_j = 0 there is no
// objective substitution.
//
// Runs at the end of a propagation round, on the state after the round's
// decisions: candidates (columns flagged when they came down to one row, and
// every column in the first round) pick the lowest candidate per row; the
// picked rows are counted, scanned and emitted in row order after the
// round's other records; then one wavefront per removed row takes it out of
// its other columns. Rows removed here make new candidates only for the next
// round.
#include "psl_kern.h"
#include "sweep.h"

namespace psl {

// the LP stopped (infeasible or unbounded, this round or before) or is done
// (in a batch, lp_ok is cleared for both)
__device__ __forceinline__ bool lp_stopped(const Dev& d, int lp) {
  if (d.K > 1) return d.lp_ok[lp] == 0;
  return (d.flags->infeasible | d.flags->unbounded) != 0;
}

__global__ void k_fs_pick(Dev d) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n || !d.fs_flag[j]) return;
  d.fs_flag[j] = 0;
  double2 b = d.bnd[j];
  if (b.x == b.y || d.col_len[j] != 1 || d.c[j] != 0.0) return;
  if (lp_stopped(d, col_lp_of(d, (int)j))) return;
  // its one alive row
  int i = -1;
  for (int q = d.cp[j]; q < d.cp[j + 1]; ++q) {
    int r = d.ri[q];
    if (d.row_on[r]) {
      i = r;
      break;
    }
  }
  if (i < 0) return;
  bool lo_ok = is_inf(b.x) || d.lsrc[j] == i;
  bool up_ok = is_inf(b.y) || d.usrc[j] == i;
  if (lo_ok && up_ok) atomicMin(&d.fs_pick[i], (int)j);
}

__global__ void k_fs_count(Dev d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) d.flags->fs_rows = 0;
  if (i < d.m) d.cnt[i] = d.fs_pick[i] != 0x7FFFFFFF;
}

// coefficient of column j in row i (columns ascend within a row)
__device__ __forceinline__ double coef_of(const Dev& d, int i, int j) {
  int lo = d.rp[i], hi = d.rp[i + 1] - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (d.ci[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return d.va[lo];
}

// rows of at most this many entries leave their columns in the emitting
// thread; longer ones are listed in chunks of FS_CHUNK positions, one
// workgroup each
#define FS_SHORT 32
#define FS_CHUNK PSL_BLOCK

// records after the round's decision records; the row leaves, the column is
// set to lb = ub = 0 (its cost is 0, so it adds nothing to the objective),
// and a short row leaves its other active columns here (no other row of this
// pass holds column j: it had one alive row)
__global__ void k_fs_emit(Dev d, int32_t* list, int64_t base, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.m) return;
  int i = (int)t;
  int j = d.fs_pick[i];
  if (j == 0x7FFFFFFF) return;
  d.fs_pick[i] = 0x7FFFFFFF;
  int lp = row_lp_of(d, i);
  Record r;
  r.type = REC_FREE_SINGLETON;
  r.side = 0;
  r.round = (uint16_t)round_of(d, lp, round);
  r.i = i;
  r.j = j;
  r.k = -1;
  r.v[0] = coef_of(d, i, j);
  r.v[1] = d.lhs[i];
  r.v[2] = d.rhs[i];
  r.v[3] = 0.0;
  d.rec[base + d.flags->round_total + d.off[t]] = r;
  d.row_on[i] = 0;
  d.bnd[j] = make_double2(0.0, 0.0);
  d.bkey[2 * (int64_t)j] = dkey(0.0);
  d.bkey[2 * (int64_t)j + 1] = dkey(0.0);
  if (d.K > 1) d.lpo[lp].total = 1;  // the LP changed this round
  int p0 = d.rp[i], len = d.rp[i + 1] - p0;
  if (len > FS_SHORT) {
    int nch = (len + FS_CHUNK - 1) / FS_CHUNK;
    int c0 = atomicAdd(&d.flags->fs_rows, nch);
    for (int c = 0; c < nch; ++c) list[c0 + c] = p0 + c * FS_CHUNK;
    return;
  }
  double lhs = r.v[1], rhs = r.v[2];
  // groups of four entries: their loads in flight together, then the drops
#pragma unroll 1
  for (int g = 0; g < len; g += 4) {
    int jj[4];
    double a[4];
    double2 bb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int p = p0 + (g + k < len ? g + k : 0);
      jj[k] = d.ci[p];
      a[k] = d.va[p];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) bb[k] = jj[k] == j ? make_double2(0.0, 0.0) : d.bnd[jj[k]];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (g + k < len && bb[k].x != bb[k].y) drop_col(d, jj[k], a[k], lhs, rhs);
  }
}

// the listed chunks of long removed rows leave their other active columns:
// one workgroup per chunk (its first CSR position listed), a position a thread
__global__ void __launch_bounds__(PSL_BLOCK) k_fs_drop(Dev d, const int32_t* list) {
  int nc = d.flags->fs_rows;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.flags->round_total += d.flags->fs_total;
    d.flags->rows_removed += d.flags->fs_total;
  }
  for (int k = blockIdx.x; k < nc; k += gridDim.x) {
    int p0 = list[k];
    int i = d.rowid1[p0 + 1];
    int p = p0 + (int)threadIdx.x;
    if (p < d.rp[i + 1]) {
      int j = d.ci[p];
      double2 b = d.bnd[j];
      if (b.x != b.y) drop_col(d, j, d.va[p], d.lhs[i], d.rhs[i]);
    }
  }
}

void launch_free_singletons(const Dev& d, int32_t* list, int64_t base, int round, int32_t* ws, hipStream_t s) {
  if (d.m == 0 || d.n == 0) return;
  hipLaunchKernelGGL(k_fs_pick, dim3((unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d);
  unsigned rb = (unsigned)((d.m + PSL_BLOCK - 1) / PSL_BLOCK);
  hipLaunchKernelGGL(k_fs_count, dim3(rb), dim3(PSL_BLOCK), 0, s, d);
  scan_excl(d.cnt, d.off, d.m, &d.flags->fs_total, ws, s);
  hipLaunchKernelGGL(k_fs_emit, dim3(rb), dim3(PSL_BLOCK), 0, s, d, list, base, round);
  hipLaunchKernelGGL(k_fs_drop, dim3(1024), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)list);
}

}  // namespace psl
