// doubleton.hip -- doubleton-equality substitution (section 2.1,
// "Explorers": an equality with two nonzeros eliminates one of its
// variables; "Postsolver": the record keeps what recovers it).
//
// Once per outer cycle, after the parallel passes. Candidates: alive rows of
// LPs still presolving with lhs = rhs (finite) and exactly two active columns
// (active lengths and removed-column constants from the pass's
// compaction-mode sweep), both |a| >= coef_tol, neither column kept by an
// earlier substitution. Row i is a_j x_j + a_k x_k = b, b = rhs - k_i. The
// eliminated column k: fewer alive rows, then larger |a|, then the lower
// index. A candidate whose rewrite of some row would cancel a coefficient to
// exactly zero is dropped. Each candidate claims its two columns and every
// alive row of column k (atomic min of the row index); it applies when it
// holds all its claims, so the applied substitutions touch disjoint rows and
// columns and the outcome does not depend on scheduling. Applying:
//   - every other alive row r of k: f = a_rk / a_k, column j gets a_rj - f a_j
//     (inserted at its sorted place when absent: the row keeps its length, the
//     entries between move by one), k's entry leaves (a dead entry, column k
//     with +0, when j was present), sides move by f b;
//   - x_k's bounds pass to x_j through (b - a_k bound) / a_j (BOUND_CHANGE from
//     row i when strictly tighter; |v| >= inf_value gives none);
//   - c_j -= (c_k / a_k) a_j; column k leaves at b / a_k with its cost (the
//     compaction's offset then gains c_k b / a_k); row i leaves.
// Records: DOUBLETON_ROW per applied row (ascending), then the transferred
// bounds per kept column (ascending, lower then upper). The transposed copy is
// rebuilt afterwards from the rewritten rows (by the caller).
//
// A row is rewritten by one lane, except a row longer than DBL_LANE_ROW that
// must take the kept column in: its entries between the two columns move by
// one, which a workgroup does afterwards in chunks (every load of a chunk
// before any of its stores).
#include <climits>

#include "psl_kern.h"
#include "sweep.h"

namespace psl {

__device__ __forceinline__ bool dbl_lp_stopped(const Dev& d, int lp) {
  if (d.K > 1) return d.lp_ok[lp] == 0;
  return (d.flags->infeasible | d.flags->unbounded) != 0;
}

__device__ __forceinline__ double dbl_side_minus(double side, double k) { return is_inf(side) ? side : pos0(side - k); }

// longest row a lane rewrites itself
#define DBL_LANE_ROW 256
#define DBL_SHIFT_BLOCK 1024
#define DBL_SHIFT_ITEMS 4

int64_t doubleton_long_cap(int64_t nnz) { return nnz / (DBL_LANE_ROW + 1) + 1; }

// position of column j among positions [s, s + len) of a row (ascending
// columns; dead entries keep their column), or -1
__device__ __forceinline__ int64_t dbl_find(const Dev& d, int64_t s, int len, int j) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (d.ci[s + mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && d.ci[s + lo] == j ? s + lo : -1;
}

__global__ void k_dbl_reset(Dev d, DblScratch S) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += stride) {
    S.cj[i] = -1;
    S.row_claim[i] = INT_MAX;
  }
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
    S.col_claim[j] = INT_MAX;
    S.by[j] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.flags->dbl_count = 0;
    d.flags->dbl_applied = 0;
    *S.long_cnt = 0;
  }
}

// candidate rows into S.list (wavefront-aggregated appends; the order of the
// list does not matter)
__global__ void k_dbl_list(Dev d, DblScratch S) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool pred = false;
  if (i < d.m)
    pred = d.row_on[i] && d.row_out[i].j == 2 && d.lhs[i] == d.rhs[i] && !is_inf(d.rhs[i]) &&
           !dbl_lp_stopped(d, row_lp_of(d, (int)i));
  unsigned long long mask = __ballot(pred);
  if (mask == 0) return;
  int lead = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane_id() == lead) base = atomicAdd(&d.flags->dbl_count, (int)__popcll(mask));
  base = __shfl(base, lead, PSL_WAVE);
  if (pred) S.list[base + __popcll(mask & lanemask_lt())] = (int)i;
}

// the first two active positions of a row (one wavefront; every lane gets them)
__device__ __forceinline__ void dbl_two_active(const Dev& d, int64_t s0, int len, int& p0, int& p1) {
  p0 = p1 = -1;
  int lane = lane_id();
  for (int q0 = 0; q0 < len && p1 < 0; q0 += PSL_WAVE) {
    int q = q0 + lane;
    bool act = false;
    if (q < len) {
      double2 b = d.bnd[d.ci[s0 + q]];
      act = b.x != b.y;
    }
    unsigned long long mask = __ballot(act);
    while (mask && p1 < 0) {
      int f = __ffsll((long long)mask) - 1;
      mask &= mask - 1;
      if (p0 < 0) p0 = q0 + f;
      else p1 = q0 + f;
    }
  }
}

// One wavefront per listed row: its two columns and the eliminated one, the
// cancellation check over the eliminated column's rows, then the claims.
__global__ void __launch_bounds__(PSL_BLOCK) k_dbl_claim(Dev d, DblScratch S) {
  int nv = d.flags->dbl_count;
  int lane = lane_id();
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int t = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); t < nv; t += wstride) {
    int i = S.list[t];
    int64_t s0 = d.rp[i];
    int len = d.rp[i + 1] - (int)s0;
    int p0, p1;
    dbl_two_active(d, s0, len, p0, p1);
    if (p1 < 0) continue;
    int j0 = d.ci[s0 + p0], j1 = d.ci[s0 + p1];
    double a0 = d.va[s0 + p0], a1 = d.va[s0 + p1];
    if (fabs(a0) < d.cfg.coef_tol || fabs(a1) < d.cfg.coef_tol || S.col_mod[j0] || S.col_mod[j1]) continue;
    int l0 = d.col_len[j0], l1 = d.col_len[j1];
    int e = l0 != l1 ? (l0 < l1 ? 0 : 1) : (fabs(a0) != fabs(a1) ? (fabs(a0) > fabs(a1) ? 0 : 1) : 0);
    int k = e ? j1 : j0, j = e ? j0 : j1;
    double ak = e ? a1 : a0, aj = e ? a0 : a1;
    bool cancel = false;
    for (int q = d.cp[k] + lane; q < d.cp[k + 1]; q += PSL_WAVE) {
      int r = d.ri[q];
      if (r == i || !d.row_on[r]) continue;
      int64_t sr = d.rp[r];
      int64_t pj = dbl_find(d, sr, d.rp[r + 1] - (int)sr, j);
      if (pj >= 0 && d.va[pj] - (d.cva[q] / ak) * aj == 0.0) cancel = true;
    }
    if (__ballot(cancel)) continue;
    if (lane == 0) {
      S.cj[i] = j;
      S.ck[i] = k;
      S.aj[i] = aj;
      S.ak[i] = ak;
      S.b[i] = dbl_side_minus(d.rhs[i], d.row_out[i].v0);
      atomicMin(&S.col_claim[j], i);
      atomicMin(&S.col_claim[k], i);
    }
    for (int q = d.cp[k] + lane; q < d.cp[k + 1]; q += PSL_WAVE) {
      int r = d.ri[q];
      if (d.row_on[r]) atomicMin(&S.row_claim[r], i);
    }
  }
}

// a candidate applies when it holds every claim it made
__global__ void __launch_bounds__(PSL_BLOCK) k_dbl_own(Dev d, DblScratch S) {
  int nv = d.flags->dbl_count;
  int lane = lane_id();
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int t = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); t < nv; t += wstride) {
    int i = S.list[t];
    int j = S.cj[i];
    if (j < 0) continue;
    int k = S.ck[i];
    bool lost = S.col_claim[j] != i || S.col_claim[k] != i;
    for (int q = d.cp[k] + lane; q < d.cp[k + 1] && !lost; q += PSL_WAVE) {
      int r = d.ri[q];
      if (d.row_on[r] && S.row_claim[r] != i) lost = true;
    }
    if (__ballot(lost) && lane == 0) S.cj[i] = -1;
  }
}

__global__ void k_dbl_count_rows(Dev d, DblScratch S) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < d.m) d.cnt[t] = S.cj[t] >= 0;
}

// DOUBLETON_ROW records in row order; the interval x_k's bounds give x_j
__global__ void k_dbl_emit_rows(Dev d, DblScratch S, int64_t base, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.m) return;
  int i = (int)t;
  int j = S.cj[i];
  if (j < 0) return;
  int k = S.ck[i];
  int lp = row_lp_of(d, i);
  double aj = S.aj[i], ak = S.ak[i], b = S.b[i];
  Record r;
  r.type = REC_DOUBLETON_ROW;
  r.side = 0;
  r.round = (uint16_t)round_of(d, lp, round);
  r.i = i;
  r.j = j;
  r.k = k;
  r.v[0] = aj;
  r.v[1] = ak;
  r.v[2] = b;
  r.v[3] = d.c[k];
  d.rec[base + d.flags->round_total + d.off[t]] = r;
  // x_j = (b - a_k x_k) / a_j decreases in x_k when a_k / a_j > 0
  double2 bk = d.bnd[k];
  bool dec = (ak > 0) == (aj > 0);
  double from_lb = is_inf(bk.x) ? (dec ? __builtin_inf() : -__builtin_inf()) : pos0((b - ak * bk.x) / aj);
  double from_ub = is_inf(bk.y) ? (dec ? -__builtin_inf() : __builtin_inf()) : pos0((b - ak * bk.y) / aj);
  double lo = dec ? from_ub : from_lb, hi = dec ? from_lb : from_ub;
  if (fabs(lo) >= d.cfg.inf_value) lo = -__builtin_inf();
  if (fabs(hi) >= d.cfg.inf_value) hi = __builtin_inf();
  S.tb[j] = make_double2(lo, hi);
  S.by[j] = i;
  atomicOr(&d.flags->dbl_applied, 1);
  d.flags->merged = 1;
  if (d.K > 1) d.lpf[lp].merged = 1;
}

__global__ void k_dbl_count_cols(Dev d, DblScratch S) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  int c = 0;
  if (S.by[j] >= 0) {
    double2 b = d.bnd[j], t = S.tb[j];
    c = (t.x > b.x ? 1 : 0) + (t.y < b.y ? 1 : 0);
  }
  d.cnt[j] = c;
}

// the transferred bounds in column order (lower, then upper), from row i
__global__ void k_dbl_emit_cols(Dev d, DblScratch S, const int32_t* row_total, int64_t base, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.n) return;
  int j = (int)t;
  int i = S.by[j];
  if (i < 0) return;
  int lp = col_lp_of(d, j);
  double2 b = d.bnd[j], tb = S.tb[j];
  double aj = S.aj[i];
  int64_t pos = base + d.flags->round_total + *row_total + d.off[t];
  double lo = b.x, up = b.y;
  Record r;
  r.round = (uint16_t)round_of(d, lp, round);
  r.type = REC_BOUND_CHANGE;
  r.i = -1;
  r.j = j;
  r.k = i;
  r.v[3] = 0.0;
  if (tb.x > b.x) {
    r.side = 0;
    r.v[0] = b.x;
    r.v[1] = tb.x;
    r.v[2] = aj;
    d.rec[pos++] = r;
    lo = tb.x;
    int ls = d.lsrc[j];
    d.lsrc[j] = ls == -1 || ls == i ? i : -2;
  }
  if (tb.y < b.y) {
    r.side = 1;
    r.v[0] = b.y;
    r.v[1] = tb.y;
    r.v[2] = aj;
    d.rec[pos++] = r;
    up = tb.y;
    int us = d.usrc[j];
    d.usrc[j] = us == -1 || us == i ? i : -2;
  }
  d.bnd[j] = make_double2(lo, up);
  d.bkey[2 * (int64_t)j] = dkey(lo);
  d.bkey[2 * (int64_t)j + 1] = dkey(up);
  d.touch[j] = 1;
  if (d.cfg.free_sing) d.fs_flag[j] = 1;
  if (!is_inf(lo) && !is_inf(up) && lo > up + tol_of(d.cfg, up)) flag_infeasible(d, lp);
}

__global__ void k_dbl_close(Dev d, const int32_t* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) d.flags->round_total += total[0] + total[1];
}

// Row r loses column k and gets v on column j, in place (one lane): see the
// header. Returns 1 when j was inserted.
__device__ __forceinline__ int dbl_rewrite(const Dev& d, int r, int k, int j, double v) {
  int64_t s = d.rp[r];
  int len = d.rp[r + 1] - (int)s;
  int64_t pk = dbl_find(d, s, len, k), pj = dbl_find(d, s, len, j);
  if (pk < 0) return 0;  // cannot happen: r came from column k's transposed copy
  int32_t* ci = const_cast<int32_t*>(d.ci);
  double* va = const_cast<double*>(d.va);
  if (pj >= 0) {
    va[pj] = v;
    va[pk] = 0.0;
    return 0;
  }
  int64_t q = pk;
  if (j > k) {
    while (q + 1 < s + len && ci[q + 1] < j) {
      ci[q] = ci[q + 1];
      va[q] = va[q + 1];
      ++q;
    }
  } else {
    while (q > s && ci[q - 1] > j) {
      ci[q] = ci[q - 1];
      va[q] = va[q - 1];
      --q;
    }
  }
  ci[q] = j;
  va[q] = v;
  return 1;
}

// One wavefront per applied substitution: the eliminated column's other
// rows (one lane each), then the costs, column k and row i.
__global__ void __launch_bounds__(PSL_BLOCK) k_dbl_apply(Dev d, DblScratch S) {
  int nv = d.flags->dbl_count;
  int lane = lane_id();
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int t = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); t < nv; t += wstride) {
    int i = S.list[t];
    int j = S.cj[i];
    if (j < 0) continue;
    int k = S.ck[i];
    double aj = S.aj[i], ak = S.ak[i], b = S.b[i];
    for (int q = d.cp[k] + lane; q < d.cp[k + 1]; q += PSL_WAVE) {
      int r = d.ri[q];
      if (r == i || !d.row_on[r]) continue;
      double f = d.cva[q] / ak;
      int64_t sr = d.rp[r];
      int len = d.rp[r + 1] - (int)sr;
      int64_t pj = dbl_find(d, sr, len, j);
      double v = (pj >= 0 ? d.va[pj] : 0.0) - f * aj;
      double sh = f * b;
      d.lhs[r] = dbl_side_minus(d.lhs[r], sh);
      d.rhs[r] = dbl_side_minus(d.rhs[r], sh);
      if (pj < 0 && len > DBL_LANE_ROW) {
        // the insertion moves up to the whole row: left to a workgroup
        DblTask tk;
        tk.r = r;
        tk.k = k;
        tk.j = j;
        tk.pad = 0;
        tk.v = v;
        S.long_task[atomicAdd(S.long_cnt, 1)] = tk;
        atomicAdd(&d.col_len[j], 1);
      } else if (dbl_rewrite(d, r, k, j, v)) {
        atomicAdd(&d.col_len[j], 1);
      }
    }
    if (lane == 0) {
      double rc = d.c[k] / ak;
      d.c[j] = pos0(d.c[j] - rc * aj);
      S.col_mod[j] = 1;
      double lhs = d.lhs[i], rhs = d.rhs[i];
      d.row_on[i] = 0;
      drop_col(d, j, aj, lhs, rhs);
      drop_col(d, k, ak, lhs, rhs);
      double vk = pos0(b / ak);
      d.bnd[k] = make_double2(vk, vk);
      d.bkey[2 * (int64_t)k] = dkey(vk);
      d.bkey[2 * (int64_t)k + 1] = dkey(vk);
    }
  }
}

// The deferred long-row insertions (one workgroup each, grid-striding): the
// entries strictly between column k's position and the kept column's sorted
// place move by one towards k's position, then j takes the freed place, as a
// lane's rewrite does. Chunks of DBL_SHIFT_BLOCK * DBL_SHIFT_ITEMS entries go
// away from k's position; a chunk's loads all precede its stores (a barrier),
// and the next chunk stores only after its own barrier, so no entry is
// overwritten before it is read.
__global__ void __launch_bounds__(DBL_SHIFT_BLOCK) k_dbl_shift(Dev d, DblScratch S) {
  __shared__ int64_t sh_pk, sh_q;
  int nt = *S.long_cnt;
  int32_t* ci = const_cast<int32_t*>(d.ci);
  double* va = const_cast<double*>(d.va);
  const int C = DBL_SHIFT_BLOCK * DBL_SHIFT_ITEMS;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    DblTask tk = S.long_task[t];
    int64_t s = d.rp[tk.r];
    int len = d.rp[tk.r + 1] - (int)s;
    if (threadIdx.x == 0) {
      sh_pk = dbl_find(d, s, len, tk.k);
      // the first position whose column exceeds j (j is absent)
      int lo = 0, hi = len;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (d.ci[s + mid] < tk.j) lo = mid + 1;
        else hi = mid;
      }
      sh_q = s + lo;
    }
    __syncthreads();
    int64_t pk = sh_pk, ub = sh_q;
    // j > k: entries (pk, ub) move down by one, j lands at ub - 1;
    // j < k: entries [ub, pk) move up by one, j lands at ub
    bool down = tk.j > tk.k;
    int64_t a = down ? pk + 1 : ub, e = down ? ub : pk;  // sources [a, e)
    int64_t L = e - a;
    for (int64_t c0 = 0; c0 < L; c0 += C) {
      int32_t cv[DBL_SHIFT_ITEMS];
      double vv[DBL_SHIFT_ITEMS];
      int64_t src[DBL_SHIFT_ITEMS];
#pragma unroll
      for (int u = 0; u < DBL_SHIFT_ITEMS; ++u) {
        int64_t o = c0 + u * DBL_SHIFT_BLOCK + threadIdx.x;  // offset from the end nearest k
        src[u] = o < L ? (down ? a + o : e - 1 - o) : -1;
        if (src[u] >= 0) {
          cv[u] = ci[src[u]];
          vv[u] = va[src[u]];
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < DBL_SHIFT_ITEMS; ++u)
        if (src[u] >= 0) {
          int64_t dst = down ? src[u] - 1 : src[u] + 1;
          ci[dst] = cv[u];
          va[dst] = vv[u];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t q = down ? ub - 1 : ub;
      ci[q] = tk.j;
      va[q] = tk.v;
    }
    __syncthreads();  // sh_pk, sh_q are set again for the next task
  }
}

// with dual fixing: a kept column's locks counted again over its alive rows
// (its coefficients changed), after the transposed copy is rebuilt
__global__ void k_dbl_relock(Dev d, DblScratch S) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n || S.by[j] < 0) return;
  unsigned long long lk = 0;
  for (int q = d.cp[j]; q < d.cp[j + 1]; ++q) {
    int r = d.ri[q];
    if (d.row_on[r] && d.cva[q] != 0.0) lk += lock_bits(d.cva[q], d.lhs[r], d.rhs[r]);
  }
  d.locks[j] = lk;
}

__global__ void k_dbl_init(Dev d, DblScratch S) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) S.col_mod[j] = 0;
}

// ---------------------------------------------------------------------------
void launch_doubleton_init(const Dev& d, const DblScratch& S, hipStream_t s) {
  if (d.n == 0) return;
  int64_t b = (d.n + PSL_BLOCK - 1) / PSL_BLOCK;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_dbl_init, dim3((unsigned)b), dim3(PSL_BLOCK), 0, s, d, S);
}

void launch_doubletons(const Dev& d, const DblScratch& S, int64_t base, int round, int32_t* ws, hipStream_t s) {
  int64_t span = d.m > d.n ? d.m : d.n;
  int64_t rb = (span + PSL_BLOCK - 1) / PSL_BLOCK;
  if (rb > 8192) rb = 8192;
  if (rb < 1) rb = 1;
  hipLaunchKernelGGL(k_dbl_reset, dim3((unsigned)rb), dim3(PSL_BLOCK), 0, s, d, S);
  if (d.m > 0) {
    unsigned mb = (unsigned)((d.m + PSL_BLOCK - 1) / PSL_BLOCK);
    hipLaunchKernelGGL(k_dbl_list, dim3(mb), dim3(PSL_BLOCK), 0, s, d, S);
    hipLaunchKernelGGL(k_dbl_claim, dim3(2048), dim3(PSL_BLOCK), 0, s, d, S);
    hipLaunchKernelGGL(k_dbl_own, dim3(2048), dim3(PSL_BLOCK), 0, s, d, S);
    hipLaunchKernelGGL(k_dbl_count_rows, dim3(mb), dim3(PSL_BLOCK), 0, s, d, S);
    scan_excl(d.cnt, d.off, d.m, S.total, ws, s);
    hipLaunchKernelGGL(k_dbl_emit_rows, dim3(mb), dim3(PSL_BLOCK), 0, s, d, S, base, round);
  } else {
    fill_i32(S.total, 0, 1, s);
  }
  if (d.n > 0) {
    unsigned nb = (unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK);
    hipLaunchKernelGGL(k_dbl_count_cols, dim3(nb), dim3(PSL_BLOCK), 0, s, d, S);
    scan_excl(d.cnt, d.off, d.n, S.total + 1, ws, s);
    hipLaunchKernelGGL(k_dbl_emit_cols, dim3(nb), dim3(PSL_BLOCK), 0, s, d, S, (const int32_t*)S.total, base, round);
  } else {
    fill_i32(S.total + 1, 0, 1, s);
  }
  hipLaunchKernelGGL(k_dbl_close, dim3(1), dim3(64), 0, s, d, (const int32_t*)S.total);
  if (d.m > 0) {
    hipLaunchKernelGGL(k_dbl_apply, dim3(2048), dim3(PSL_BLOCK), 0, s, d, S);
    hipLaunchKernelGGL(k_dbl_shift, dim3(256), dim3(DBL_SHIFT_BLOCK), 0, s, d, S);
  }
}

void launch_doubleton_relock(const Dev& d, const DblScratch& S, hipStream_t s) {
  if (d.n == 0 || !d.cfg.dual_fix) return;
  hipLaunchKernelGGL(k_dbl_relock, dim3((unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d,
                     S);
}

}  // namespace psl
