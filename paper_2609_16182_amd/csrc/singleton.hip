// singleton.hip -- elimination of free column singletons (section 3.2,
// "Column singletons"): a column in one alive row i, whose bounds are
// infinite or were tightened only from row i (so they are implied by it), can
// take any value row i needs; row i and the column leave together and
// postsolve recovers x_j from the row. A column with a cost is substituted
// into the objective: with r = c_j / a_ij the row's activity goes to the side
// the cost prefers (r > 0: lhs, r < 0: rhs; an infinite one makes the LP
// unbounded if feasible), every other cost of the row becomes c_k - r a_ik
// and the column is kept at s / a_ij with its cost, which puts r s into the
// objective offset.
//
// Runs at the end of a propagation round, on the state after the round's
// decisions. Candidates (columns flagged when they came down to one row, and
// every column in the first round) pick the lowest candidate per row. Rows
// whose column has a cost claim all their columns (an atomic min of a key of
// the round and the row, so the previous rounds' claims need no clearing);
// such a row applies only where it is the lowest claimant of each column, so
// no cost changes twice in a round (the others wait for the next round). The
// applying rows are counted, scanned and emitted in row order after the
// round's other records; rows of at most FS_SHORT entries update costs and
// leave their columns in their own thread, longer ones are deferred to lists
// of FS_CHUNK-position chunks, one workgroup each. Rows removed here make
// new candidates only for the next round.
#include "psl_kern.h"
#include "sweep.h"

namespace psl {

#define FS_SHORT 32
#define FS_CHUNK PSL_BLOCK
#define FS_NONE 0x7FFFFFFF

// the LP stopped (infeasible or unbounded, this round or before) or is done
// (in a batch, lp_ok is cleared for both)
__device__ __forceinline__ bool lp_stopped(const Dev& d, int lp) {
  if (d.K > 1) return d.lp_ok[lp] == 0;
  return (d.flags->infeasible | d.flags->unbounded) != 0;
}

// the column's one alive row i takes the column when each bound side is
// infinite or was tightened only from row i
__device__ __forceinline__ void fs_offer(const Dev& d, int j, int i) {
  double2 b = d.bnd[j];
  bool lo_ok = is_inf(b.x) || d.lsrc[j] == i;
  bool up_ok = is_inf(b.y) || d.usrc[j] == i;
  if (lo_ok && up_ok) atomicMin(&d.fs_pick[i], j);
}

// flagged columns of length 1 find their alive row on the transposed copy:
// columns stored with at most FS_PICK_SHORT entries in their own lane, longer
// ones (a dense column down to one row) by the whole wavefront, one after
// another, 64 positions a step
#define FS_PICK_SHORT 64
__global__ void __launch_bounds__(PSL_BLOCK) k_fs_pick(Dev d) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) d.flags->fs_claims = 0;
  bool want = false;
  if (j < d.n && d.fs_flag[j]) {
    d.fs_flag[j] = 0;
    double2 b = d.bnd[j];
    want = b.x != b.y && d.col_len[j] == 1 && !lp_stopped(d, col_lp_of(d, (int)j));
  }
  int q0 = 0, q1 = 0;
  if (want) {
    q0 = d.cp[j];
    q1 = d.cp[j + 1];
  }
  bool longc = want && q1 - q0 > FS_PICK_SHORT;
  if (want && !longc) {
    for (int q = q0; q < q1; ++q) {
      int r = d.ri[q];
      if (d.row_on[r]) {
        fs_offer(d, (int)j, r);
        break;
      }
    }
  }
  unsigned long long mask = __ballot(longc);
  int lane = lane_id();
  while (mask) {
    int l = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    int jl = __shfl((int)j, l, PSL_WAVE), a = __shfl(q0, l, PSL_WAVE), e = __shfl(q1, l, PSL_WAVE);
    for (int base = a; base < e; base += PSL_WAVE) {
      int q = base + lane;
      int r = q < e ? d.ri[q] : -1;
      unsigned long long hit = __ballot(r >= 0 && d.row_on[r]);
      if (hit) {  // the same on every lane
        int i = __shfl(r, __ffsll((long long)hit) - 1, PSL_WAVE);
        if (lane == 0) fs_offer(d, jl, i);
        break;
      }
    }
  }
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

// append the chunks of a row (positions p0 .. p0 + len) to a chunk list
__device__ __forceinline__ void list_chunks(int32_t* list, int32_t* count, int p0, int len) {
  int nch = (len + FS_CHUNK - 1) / FS_CHUNK;
  int c0 = atomicAdd(count, nch);
  for (int c = 0; c < nch; ++c) list[c0 + c] = p0 + c * FS_CHUNK;
}

// the claim of row i in a round: claims of the round compare by row, and any
// of them is below a claim left from an earlier round of the run
__device__ __forceinline__ unsigned long long fs_key(int round, int i) {
  return ((unsigned long long)(0xFFFFFFFFu - (unsigned)round) << 32) | (unsigned)i;
}

// rows whose column has a cost: an infinite preferred side stops the LP;
// otherwise they claim their columns (long rows through the claim list)
__global__ void k_fs_claim(Dev d, int32_t* clist, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.m) return;
  int i = (int)t;
  int j = d.fs_pick[i];
  if (j == FS_NONE) return;
  d.fs_bad[i] = 0;
  double cj = d.c[j];
  if (cj == 0.0) return;
  double r = cj / coef_of(d, i, j);
  if (is_inf(r > 0 ? d.lhs[i] : d.rhs[i])) {
    flag_unbounded(d, row_lp_of(d, i));
    return;
  }
  int p0 = d.rp[i], len = d.rp[i + 1] - p0;
  if (len > FS_SHORT) {
    list_chunks(clist, &d.flags->fs_claims, p0, len);
    return;
  }
  unsigned long long key = fs_key(round, i);
  for (int p = p0; p < p0 + len; ++p) atomicMin(&d.owner[d.ci[p]], key);
}

// chunks of long claiming rows: MODE 0 claims the columns, MODE 1 marks the
// row when a lower row holds one of them
template <int MODE>
__global__ void __launch_bounds__(PSL_BLOCK) k_fs_claim_long(Dev d, const int32_t* clist, int round) {
  int nc = d.flags->fs_claims;
  for (int k = blockIdx.x; k < nc; k += gridDim.x) {
    int p0 = clist[k];
    int i = d.rowid1[p0 + 1];
    int p = p0 + (int)threadIdx.x;
    if (p < d.rp[i + 1]) {
      unsigned long long key = fs_key(round, i);
      if (MODE == 0) atomicMin(&d.owner[d.ci[p]], key);
      else if (d.owner[d.ci[p]] != key) d.fs_bad[i] = 1;
    }
  }
}

// a row applies when its LP goes on and, with a cost, it holds every column
__device__ __forceinline__ bool fs_applies(const Dev& d, int i, int j, int round) {
  if (lp_stopped(d, row_lp_of(d, i))) return false;
  if (d.c[j] == 0.0) return true;
  int p0 = d.rp[i], len = d.rp[i + 1] - p0;
  if (len > FS_SHORT) return d.fs_bad[i] == 0;
  unsigned long long key = fs_key(round, i);
  for (int p = p0; p < p0 + len; ++p)
    if (d.owner[d.ci[p]] != key) return false;
  return true;
}

// applying rows keep their pick, the others drop it; d.cnt gets the count
// of each tile of PSL_BLOCK rows
__global__ void __launch_bounds__(PSL_BLOCK) k_fs_count(Dev d, int round) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) d.flags->fs_rows = 0;
  int k = 0;
  if (i < d.m) {
    int j = d.fs_pick[i];
    if (j != FS_NONE) {
      if (fs_applies(d, (int)i, j, round)) {
        k = 1;
      } else {  // waits for the next round: its column is checked again then
        d.fs_pick[i] = FS_NONE;
        d.fs_flag[j] = 1;
      }
    }
  }
  int tot;
  block_excl_scan(k, &tot);
  if (threadIdx.x == 0) d.cnt[blockIdx.x] = tot;
}

// the other columns of an applying row: a new cost (with a substitution) and
// the row's leaving (active columns); no other applying row holds them
__device__ __forceinline__ void fs_entry(const Dev& d, int jj, double a, double2 b, bool subst, double r, double lhs,
                                         double rhs) {
  if (subst) {
    d.c[jj] = pos0(d.c[jj] - r * a);
    d.touch[jj] = 1;  // its cost changed: decided again next round
  }
  if (b.x != b.y) drop_col(d, jj, a, lhs, rhs);
}

// records after the round's decision records, in row order (tile offsets
// from the scanned tile counts, a block scan inside the tile); the row
// leaves, its column is set to s / a_ij (0 without a cost); a short row
// updates and leaves its other columns here, a long one is listed in chunks
// (and keeps its pick for them)
__global__ void __launch_bounds__(PSL_BLOCK) k_fs_emit(Dev d, int32_t* list, int64_t base, int round) {
  if (d.cnt[blockIdx.x] == 0) return;  // no row of the tile applies
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int j = t < d.m ? d.fs_pick[t] : FS_NONE;
  int tot;
  int pre = block_excl_scan(j != FS_NONE ? 1 : 0, &tot);
  if (j == FS_NONE) return;
  int i = (int)t;
  int lp = row_lp_of(d, i);
  double a = coef_of(d, i, j), cj = d.c[j];
  double lhs = d.lhs[i], rhs = d.rhs[i];
  double r = cj / a;
  int side = cj == 0.0 ? 0 : (r > 0 ? 1 : 2);
  double v = side == 0 ? 0.0 : pos0((side == 1 ? lhs : rhs) / a);
  Record rec;
  rec.type = REC_FREE_SINGLETON;
  rec.side = (uint8_t)side;
  rec.round = (uint16_t)round_of(d, lp, round);
  rec.i = i;
  rec.j = j;
  rec.k = -1;
  rec.v[0] = a;
  rec.v[1] = lhs;
  rec.v[2] = rhs;
  rec.v[3] = cj;
  d.rec[base + d.flags->round_total + d.off[blockIdx.x] + pre] = rec;
  d.row_on[i] = 0;
  d.bnd[j] = make_double2(v, v);
  d.bkey[2 * (int64_t)j] = dkey(v);
  d.bkey[2 * (int64_t)j + 1] = dkey(v);
  if (d.K > 1) d.lpo[lp].total = 1;  // the LP changed this round
  int p0 = d.rp[i], len = d.rp[i + 1] - p0;
  if (len > FS_SHORT) {
    list_chunks(list, &d.flags->fs_rows, p0, len);
    return;
  }
  d.fs_pick[i] = FS_NONE;
  // groups of four entries: their loads in flight together, then the updates
#pragma unroll 1
  for (int g = 0; g < len; g += 4) {
    int jj[4];
    double aa[4];
    double2 bb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int p = p0 + (g + k < len ? g + k : 0);
      jj[k] = d.ci[p];
      aa[k] = d.va[p];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) bb[k] = jj[k] == j ? make_double2(v, v) : d.bnd[jj[k]];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (g + k < len && jj[k] != j) fs_entry(d, jj[k], aa[k], bb[k], side != 0, r, lhs, rhs);
  }
}

// the listed chunks of long applying rows: one workgroup per chunk, a
// position a thread (the row's own column was set at its emission)
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
    if (p >= d.rp[i + 1]) continue;
    int j = d.fs_pick[i];
    int jj = d.ci[p];
    if (jj == j) continue;
    double cj = d.c[j];
    double r = cj / coef_of(d, i, j);
    fs_entry(d, jj, d.va[p], d.bnd[jj], cj != 0.0, r, d.lhs[i], d.rhs[i]);
  }
}

// the long rows' picks, once all their chunks are done
__global__ void k_fs_reset(Dev d, const int32_t* list) {
  int nc = d.flags->fs_rows;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += gridDim.x * blockDim.x) {
    int p0 = list[k];
    int i = d.rowid1[p0 + 1];
    if (p0 == d.rp[i]) d.fs_pick[i] = FS_NONE;  // the row's first chunk
  }
}

void launch_free_singletons(const Dev& d, int32_t* list, int64_t base, int round, int32_t* ws, hipStream_t s) {
  if (d.m == 0 || d.n == 0) return;
  // the claim chunks follow the room of the drop chunks (at most nnz / FS_SHORT
  // + m of each)
  int32_t* clist = list + (d.nnz / FS_SHORT + d.m + 64);
  unsigned cb = (unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK);
  unsigned rb = (unsigned)((d.m + PSL_BLOCK - 1) / PSL_BLOCK);
  hipLaunchKernelGGL(k_fs_pick, dim3(cb), dim3(PSL_BLOCK), 0, s, d);
  hipLaunchKernelGGL(k_fs_claim, dim3(rb), dim3(PSL_BLOCK), 0, s, d, clist, round);
  hipLaunchKernelGGL((k_fs_claim_long<0>), dim3(1024), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)clist, round);
  hipLaunchKernelGGL((k_fs_claim_long<1>), dim3(1024), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)clist, round);
  hipLaunchKernelGGL(k_fs_count, dim3(rb), dim3(PSL_BLOCK), 0, s, d, round);
  // tile counts (rb <= m entries of d.cnt) scanned
  scan_excl(d.cnt, d.off, rb, &d.flags->fs_total, ws, s);
  hipLaunchKernelGGL(k_fs_emit, dim3(rb), dim3(PSL_BLOCK), 0, s, d, list, base, round);
  hipLaunchKernelGGL(k_fs_drop, dim3(1024), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)list);
  hipLaunchKernelGGL(k_fs_reset, dim3(64), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)list);
}

}  // namespace psl
