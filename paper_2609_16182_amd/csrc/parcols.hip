// parcols.hip -- parallel columns (section 3.2, "Parallel columns"): columns
// j, k with a_j = lambda a_k (over the alive rows) and c_j = lambda c_k are
// parallel rows of [c A'] and merge into one variable x_k + lambda x_j, whose
// interval is [lb_k, ub_k] + lambda [lb_j, ub_j].
//
// Candidates are the active columns in at least one alive row, of any length.
// Each gets a 63-bit key of its augmented row (the cost as an entry of id
// 2^32 - 1 before the rows, rows in the LP's own numbering, entries over the
// first one): a thread per column of at most PC_SHORT stored entries, a
// wavefront per longer one (the key is a sum modulo 2^64, so the lanes' order
// does not matter). The candidates are sorted stably by key (two LSD passes
// of four digits over the key's halves; then by LP in a batch), so that a group
// of equal keys lists its columns in ascending order. The group's first column
// leads; every other member is verified against it (a thread, or a wavefront
// when either column is long) and the head adds their scaled intervals in
// column order. Records in one pass over the columns (LEADER_BOUNDS for a
// leader, PARALLEL_COL for a merged column); a merged column is set to 0,
// since the leader carries it.
#include <utility>

#include "psl_kern.h"
#include "sweep.h"

namespace psl {

#define PC_SHORT 64
#define PC_NONE 0xFFFFFFFFFFFFFFFFull

__device__ __forceinline__ bool pc_lp_stopped(const Dev& d, int lp) {
  if (d.K > 1) return d.lp_ok[lp] == 0;
  return (d.flags->infeasible | d.flags->unbounded) != 0;
}

// first entry of the augmented row of column j (its cost, else its first
// alive coefficient)
__device__ __forceinline__ double pc_first(const Dev& d, int j) {
  if (d.c[j] != 0.0) return d.c[j];
  for (int q = d.cp[j]; q < d.cp[j + 1]; ++q)
    if (d.row_on[d.ri[q]]) return d.cva[q];
  return 0.0;
}

// the same from one wavefront (every lane returns it)
__device__ __forceinline__ double pc_first_wave(const Dev& d, int j) {
  if (d.c[j] != 0.0) return d.c[j];
  int q1 = d.cp[j + 1];
  for (int q0 = d.cp[j]; q0 < q1; q0 += PSL_WAVE) {
    int q = q0 + lane_id();
    unsigned long long m = __ballot(q < q1 && d.row_on[d.ri[q]]);
    if (m) return d.cva[q0 + __ffsll((long long)m) - 1];
  }
  return 0.0;
}

__device__ __forceinline__ bool pc_candidate(const Dev& d, int j) {
  double2 b = d.bnd[j];
  return b.x != b.y && d.col_len[j] >= 1 && !pc_lp_stopped(d, col_lp_of(d, j));
}

// the hash terms of entry q of column j (alive rows only)
__device__ __forceinline__ void pc_term(const Dev& d, int q, int row0, double f, unsigned long long& h1,
                                        unsigned long long& h2) {
  int i = d.ri[q];
  if (!d.row_on[i]) return;
  unsigned long long id = splitmix((unsigned long long)(uint32_t)(i - row0));
  h1 += 1 + id;
  h2 += splitmix(id ^ quantize(d.cva[q] / f));
}

__device__ __forceinline__ void pc_cost_term(double c, double f, unsigned long long& h1, unsigned long long& h2) {
  if (c == 0.0) return;
  unsigned long long id = splitmix(0xFFFFFFFFull);
  h1 += 1 + id;
  h2 += splitmix(id ^ quantize(c / f));
}

__device__ __forceinline__ void pc_set_key(const ColScratch& P, int j, unsigned long long key) {
  P.key[j] = key;
  P.keys[j] = (uint32_t)key;
}

// keys of the short candidates; the long ones go to a list (n_long counts it)
__global__ void k_pc_keys(Dev d, ColScratch P, int32_t* long_list, int32_t* n_long) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.n) return;
  int j = (int)t;
  P.lead[j] = -1;
  P.vals[j] = j;
  unsigned long long key = PC_NONE;
  if (pc_candidate(d, j)) {
    int q0 = d.cp[j], q1 = d.cp[j + 1];
    if (q1 - q0 > PC_SHORT) {
      long_list[atomicAdd(n_long, 1)] = j;
      return;  // keyed by k_pc_keys_long
    }
    int lp = col_lp_of(d, j);
    int row0 = d.K > 1 ? d.lp_row0[lp] : 0;
    double f = pc_first(d, j);
    unsigned long long h1 = 0, h2 = 0;
    pc_cost_term(d.c[j], f, h1, h2);
    for (int q = q0; q < q1; ++q) pc_term(d, q, row0, f, h1, h2);
    key = (splitmix(h1) ^ h2) >> 1;
  }
  pc_set_key(P, j, key);
}

// keys of the long candidates, one wavefront each
__global__ void __launch_bounds__(PSL_BLOCK) k_pc_keys_long(Dev d, ColScratch P, const int32_t* long_list,
                                                             const int32_t* n_long) {
  int nl = *n_long;
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int w = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); w < nl; w += wstride) {
    int j = long_list[w];
    int lp = col_lp_of(d, j);
    int row0 = d.K > 1 ? d.lp_row0[lp] : 0;
    double f = pc_first_wave(d, j);
    unsigned long long h1 = 0, h2 = 0;
    if (lane_id() == 0) pc_cost_term(d.c[j], f, h1, h2);
    int q1 = d.cp[j + 1];
    for (int q = d.cp[j] + lane_id(); q < q1; q += PSL_WAVE) pc_term(d, q, row0, f, h1, h2);
    h1 = group_sum_u64<PSL_WAVE>(h1);
    h2 = group_sum_u64<PSL_WAVE>(h2);
    if (lane_id() == 0) pc_set_key(P, j, (splitmix(h1) ^ h2) >> 1);
  }
}

// the high halves of the keys in the order of the sort by the low halves
__global__ void k_pc_hikeys(Dev d, const int32_t* vals, const uint64_t* key, uint32_t* out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < d.n) out[p] = (uint32_t)(key[vals[p]] >> 32);
}

// batch: the LP of each sorted column, for the sort by LP
__global__ void k_pc_lpkeys(Dev d, const int32_t* vals, uint32_t* keys) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < d.n) keys[t] = (uint32_t)d.col_lp[vals[t]];
}

// same augmented pattern and entries within par_tol after normalisation
__device__ bool pc_parallel(const Dev& d, int j, int k, double fj, double fk) {
  if ((d.c[j] != 0.0) != (d.c[k] != 0.0)) return false;
  int qj = d.cp[j], ej = d.cp[j + 1], qk = d.cp[k], ek = d.cp[k + 1];
  for (;;) {
    while (qj < ej && !d.row_on[d.ri[qj]]) ++qj;
    while (qk < ek && !d.row_on[d.ri[qk]]) ++qk;
    bool hj = qj < ej, hk = qk < ek;
    if (hj != hk) return false;
    if (!hj) return true;
    if (d.ri[qj] != d.ri[qk]) return false;
    double a = d.cva[qj] / fj, bb = d.cva[qk] / fk;
    double scale = fabs(a) > fabs(bb) ? fabs(a) : fabs(bb);
    if (!(fabs(a - bb) <= d.cfg.par_tol * scale)) return false;
    ++qj;
    ++qk;
  }
}

__device__ __forceinline__ double pc_canon(const Cfg& c, double v) {
  if (fabs(v) >= c.inf_value) return v > 0 ? __builtin_inf() : -__builtin_inf();
  return pos0(v);
}

// kind of each sorted position: 1 the first column of a group, 0 another
// member of a group, 2 no candidate
__global__ void k_pc_heads(Dev d, const int32_t* vals, const uint64_t* key, int32_t* kind) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.n) return;
  int k = vals[p];
  uint64_t kk = key[k];
  int r = 2;
  if (kk != PC_NONE) {
    r = 1;
    if (p > 0) {
      int kp = vals[p - 1];
      if (key[kp] == kk && col_lp_of(d, kp) == col_lp_of(d, k)) r = 0;
    }
  }
  kind[p] = r;
}

// heads[g] = sorted position of the first column of group g (seg: exclusive
// scan of the head flags)
__global__ void k_pc_headpos(Dev d, const int32_t* kind, const int32_t* seg, int32_t* heads) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < d.n && kind[p] == 1) heads[seg[p]] = (int)p;
}

// a merged member's scaled interval at its sorted position (NaN: not merged)
__device__ __forceinline__ void pc_member(const Dev& d, const ColScratch& P, int64_t p, int j, int k, bool par,
                                          double fj, double fk) {
  double2 t = make_double2(__builtin_nan(""), 0.0);
  if (par) {
    double lam = fj / fk;
    double2 bj = d.bnd[j];
    t = lam > 0 ? make_double2(lam * bj.x, lam * bj.y) : make_double2(lam * bj.y, lam * bj.x);
    P.lead[j] = k;
    P.lam[j] = lam;
  }
  P.terms[p] = t;
}

// each other member against its group's first column, by a thread when both
// are short; the others go to a list (n_long counts it)
__global__ void k_pc_verify(Dev d, ColScratch P, const int32_t* vals, const int32_t* kind, const int32_t* seg,
                            const int32_t* heads, int32_t* long_list, int32_t* n_long) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.n || kind[p] != 0) return;
  int j = vals[p];
  int k = vals[heads[seg[p] - 1]];
  if (d.cp[j + 1] - d.cp[j] > PC_SHORT || d.cp[k + 1] - d.cp[k] > PC_SHORT) {
    long_list[atomicAdd(n_long, 1)] = (int)p;
    return;
  }
  double fj = pc_first(d, j), fk = pc_first(d, k);
  pc_member(d, P, p, j, k, pc_parallel(d, j, k, fj, fk), fj, fk);
}

// position of row i in column k (rows ascending), or -1
__device__ __forceinline__ int pc_find(const Dev& d, int k, int i) {
  int lo = d.cp[k], hi = d.cp[k + 1];
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (d.ri[mid] < i) lo = mid + 1;
    else hi = mid;
  }
  return lo < d.cp[k + 1] && d.ri[lo] == i ? lo : -1;
}

// the listed members, one wavefront each: parallel when both columns are in
// as many alive rows and every alive entry of the member is in the leader
// (binary search) with the same normalised value within par_tol
__global__ void __launch_bounds__(PSL_BLOCK) k_pc_verify_long(Dev d, ColScratch P, const int32_t* vals,
                                                               const int32_t* seg, const int32_t* heads,
                                                               const int32_t* long_list, const int32_t* n_long) {
  int nl = *n_long;
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int w = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); w < nl; w += wstride) {
    int64_t p = long_list[w];
    int j = vals[p];
    int k = vals[heads[seg[p] - 1]];
    double fj = pc_first_wave(d, j), fk = pc_first_wave(d, k);
    bool ok = (d.c[j] != 0.0) == (d.c[k] != 0.0) && d.col_len[j] == d.col_len[k];
    int q1 = d.cp[j + 1];
    for (int q0 = d.cp[j]; ok && q0 < q1; q0 += PSL_WAVE) {
      int q = q0 + lane_id();
      bool bad = false;
      if (q < q1 && d.row_on[d.ri[q]]) {
        int qk = pc_find(d, k, d.ri[q]);
        if (qk < 0) {
          bad = true;
        } else {
          double a = d.cva[q] / fj, bb = d.cva[qk] / fk;
          double scale = fabs(a) > fabs(bb) ? fabs(a) : fabs(bb);
          bad = !(fabs(a - bb) <= d.cfg.par_tol * scale);
        }
      }
      ok = __ballot(bad) == 0;
    }
    if (lane_id() == 0) pc_member(d, P, p, j, k, ok, fj, fk);
  }
}

// The fold of a group's member terms onto its leader's interval, members in
// column order, canonical after every add (the reference definition); the
// loads of the next PC_ACC members are issued together ahead of the adds. The
// fast path (pc_step, k_pc_accum) uses plain adds, canonical once at the end,
// and flags a partial sum that is finite with |v| >= inf_value: until then the
// two folds agree up to the sign of a zero (x + 0 = x), and an infinite term
// makes both infinite from there on (lower sums only meet -inf, upper sums
// +inf), so the results are identical unless that flag is set, and then this
// fold is run instead.
#define PC_ACC 16
__device__ __forceinline__ void pc_fold(const Dev& d, const ColScratch& P, const int32_t* kind, int64_t p, double& lo,
                                        double& up) {
  bool done = false;
  for (int64_t q = p + 1; !done; q += PC_ACC) {
    int kk[PC_ACC];
    double2 tt[PC_ACC];
#pragma unroll
    for (int b = 0; b < PC_ACC; ++b) {
      bool in = q + b < d.n;
      kk[b] = in ? kind[q + b] : 1;
      tt[b] = in ? P.terms[q + b] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int b = 0; b < PC_ACC; ++b) {
      if (done) continue;
      if (kk[b] != 0) {
        done = true;
      } else if (tt[b].x == tt[b].x) {  // NaN: not merged
        lo = pc_canon(d.cfg, lo + tt[b].x);
        up = pc_canon(d.cfg, up + tt[b].y);
      }
    }
  }
}

// lane l's value of v (l the same on every lane), through two readlanes
__device__ __forceinline__ double lane_value(double v, int l) {
  long long bits = __double_as_longlong(v);
  unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(bits & 0xFFFFFFFFll), l);
  unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// one fast-fold step over a lane's PC_ACC positions from q
__device__ __forceinline__ void pc_step(const Dev& d, const ColScratch& P, const int32_t* kind, int64_t q, double& lo,
                                        double& up, bool& any, bool& huge, bool& done) {
  double inf_v = d.cfg.inf_value;
  int kk[PC_ACC];
  double2 tt[PC_ACC];
#pragma unroll
  for (int b = 0; b < PC_ACC; ++b) {
    bool in = q + b < d.n;
    kk[b] = in ? kind[q + b] : 1;
    tt[b] = in ? P.terms[q + b] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int b = 0; b < PC_ACC; ++b) {
    if (done) continue;
    if (kk[b] != 0) {
      done = true;
    } else if (tt[b].x == tt[b].x) {
      lo = lo + tt[b].x;
      up = up + tt[b].y;
      huge = huge || (fabs(lo) >= inf_v && !is_inf(lo)) || (fabs(up) >= inf_v && !is_inf(up));
      any = true;
    }
  }
}

// The merged interval of each group. The head's lane folds the first PC_ACC
// members; a longer group is continued by the whole wavefront (groups one
// after another), 64 positions a step: coalesced loads, the group's end from a
// ballot, the next step's loads issued before this step's terms are folded
// (every lane folds them in order, reading them lane by lane). Then the
// canonical end (or the exact fold, see pc_fold) and the wrong-side check.
__global__ void __launch_bounds__(PSL_BLOCK) k_pc_accum(Dev d, ColScratch P, const int32_t* vals, const int32_t* kind) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // a head of a group of two or more
  bool head = p + 1 < d.n && kind[p] == 1 && kind[p + 1] == 0;
  int k = 0;
  double lo = 0.0, up = 0.0;
  bool any = false, huge = false, done = true;
  if (head) {
    k = vals[p];
    double2 bk = d.bnd[k];
    lo = bk.x;
    up = bk.y;
    done = false;
    pc_step(d, P, kind, p + 1, lo, up, any, huge, done);
  }
  int lane = lane_id();
  double inf_v = d.cfg.inf_value;
  unsigned long long mask = __ballot(head && !done);
  while (mask) {
    int l = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    int q = __shfl((int)p, l, PSL_WAVE) + 1 + PC_ACC;
    double glo = __shfl(lo, l, PSL_WAVE), gup = __shfl(up, l, PSL_WAVE);
    bool gany = __shfl((int)any, l, PSL_WAVE) != 0, ghuge = __shfl((int)huge, l, PSL_WAVE) != 0;
    int qq = q + lane;
    int kq = qq < d.n ? kind[qq] : 1;
    double2 t = qq < d.n ? P.terms[qq] : make_double2(0.0, 0.0);
    for (bool gdone = false; !gdone; q += PSL_WAVE) {
      unsigned long long endm = __ballot(kq != 0);
      int cnt = endm ? __ffsll((long long)endm) - 1 : PSL_WAVE;
      gdone = endm != 0;
      double2 cur = t;
      if (!gdone) {  // the next step's loads, ahead of this step's fold
        int qn = q + PSL_WAVE + lane;
        kq = qn < d.n ? kind[qn] : 1;
        t = qn < d.n ? P.terms[qn] : make_double2(0.0, 0.0);
      }
      for (int b = 0; b < cnt; ++b) {
        double tx = lane_value(cur.x, b), ty = lane_value(cur.y, b);
        if (tx == tx) {
          glo = glo + tx;
          gup = gup + ty;
          ghuge = ghuge || (fabs(glo) >= inf_v && !is_inf(glo)) || (fabs(gup) >= inf_v && !is_inf(gup));
          gany = true;
        }
      }
    }
    if (lane == l) {
      lo = glo;
      up = gup;
      any = gany;
      huge = ghuge;
    }
  }
  if (!head) return;
  lo = pc_canon(d.cfg, lo);
  up = pc_canon(d.cfg, up);
  if (huge) {  // a partial sum reached inf_value: the canonical fold itself
    double2 bk = d.bnd[k];
    lo = bk.x;
    up = bk.y;
    pc_fold(d, P, kind, p, lo, up);
  }
  if (any && (!(lo < __builtin_inf()) || !(up > -__builtin_inf()))) {
    // the merged interval passed inf_value on the wrong side: no finite value
    // would satisfy it, so the group is not merged (its members let go); a
    // lower sum at +inf that then met a -inf term is NaN (the mirror for the
    // upper sum) and is not merged either
    for (int64_t q = p + 1; q < d.n && kind[q] == 0; ++q) P.lead[vals[q]] = -1;
    any = false;
  }
  if (any) {
    P.lead[k] = k;
    P.nb[k] = make_double2(lo, up);
  }
}

__global__ void k_pc_flag1(Dev d, const int32_t* kind, int32_t* flag) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < d.n) flag[p] = kind[p] == 1;
}

__global__ void k_pc_count(Dev d, ColScratch P) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < d.n) d.cnt[j] = P.lead[j] >= 0;
}

__global__ void k_pc_emit(Dev d, ColScratch P, int64_t base, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.n) return;
  int j = (int)t;
  int k = P.lead[j];
  if (k < 0) return;
  int lp = col_lp_of(d, j);
  double2 b = d.bnd[j];
  Record r;
  r.side = 0;
  r.round = (uint16_t)round_of(d, lp, round);
  r.i = -1;
  r.j = j;
  if (k == j) {
    double2 nb = P.nb[j];
    r.type = REC_LEADER_BOUNDS;
    r.k = -1;
    r.v[0] = b.x;
    r.v[1] = b.y;
    r.v[2] = nb.x;
    r.v[3] = nb.y;
    d.bnd[j] = nb;
    d.bkey[2 * (int64_t)j] = dkey(nb.x);
    d.bkey[2 * (int64_t)j + 1] = dkey(nb.y);
    d.lsrc[j] = is_inf(nb.x) ? -1 : -2;
    d.usrc[j] = is_inf(nb.y) ? -1 : -2;
    d.touch[j] = 1;
    // an interval that became infinite can make it a free singleton: check it
    // at the next round's end
    if (d.cfg.free_sing) d.fs_flag[j] = 1;
  } else {
    r.type = REC_PARALLEL_COL;
    r.k = k;
    r.v[0] = P.lam[j];
    r.v[1] = b.x;
    r.v[2] = b.y;
    r.v[3] = 0.0;
    d.bnd[j] = make_double2(0.0, 0.0);
    d.bkey[2 * (int64_t)j] = dkey(0.0);
    d.bkey[2 * (int64_t)j + 1] = dkey(0.0);
    d.flags->merged = 1;
    if (d.K > 1) d.lpf[lp].merged = 1;
  }
  d.rec[base + d.flags->round_total + d.off[t]] = r;
}

__global__ void k_pc_close(Dev d, const int32_t* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) d.flags->round_total += *total;
}

size_t par_cols_ws_ints(int64_t n) { return radix_ws_ints(n); }

void launch_par_cols(const Dev& d, const ColScratch& P, int64_t base, int round, int32_t* ws, hipStream_t s) {
  if (d.n == 0) return;
  unsigned nb = (unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK);
  // the long candidates' list in d.cnt (free until the count pass), its
  // length in P.total
  fill_i32(P.total, 0, 1, s);
  hipLaunchKernelGGL(k_pc_keys, dim3(nb), dim3(PSL_BLOCK), 0, s, d, P, d.cnt, P.total);
  hipLaunchKernelGGL(k_pc_keys_long, dim3(1024), dim3(PSL_BLOCK), 0, s, d, P, (const int32_t*)d.cnt,
                     (const int32_t*)P.total);
  // stable LSD sort of the columns by key (63 bits; non-candidates last):
  // four passes over the low half, then four over the high half
  uint32_t* ka = P.keys;
  uint32_t* kb = P.keys2;
  int32_t* va = P.vals;
  int32_t* vb = P.vals2;
  for (int half = 0; half < 2; ++half) {
    if (half == 1)
      hipLaunchKernelGGL(k_pc_hikeys, dim3(nb), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)va, (const uint64_t*)P.key,
                         ka);
    for (int shift = 0; shift < 32; shift += 8) {
      radix_pass(ka, va, kb, vb, d.n, shift, 8, ws, s);
      std::swap(ka, kb);
      std::swap(va, vb);
    }
  }
  if (d.K > 1) {  // then by LP, keeping the key order inside an LP
    hipLaunchKernelGGL(k_pc_lpkeys, dim3(nb), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)va, ka);
    for (int shift = 0; (1ll << shift) < d.K; shift += 8) {
      radix_pass(ka, va, kb, vb, d.n, shift, 8, ws, s);
      std::swap(ka, kb);
      std::swap(va, vb);
    }
  }
  // groups: kinds (in the free key buffer), group numbers by a scan of the
  // head flags, first positions (in the free value buffer)
  int32_t* kind = reinterpret_cast<int32_t*>(ka);
  int32_t* seg = reinterpret_cast<int32_t*>(kb);
  int32_t* heads = vb;
  hipLaunchKernelGGL(k_pc_heads, dim3(nb), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)va, (const uint64_t*)P.key,
                     kind);
  hipLaunchKernelGGL(k_pc_flag1, dim3(nb), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)kind, seg);
  scan_excl(seg, seg, d.n, nullptr, ws, s);
  hipLaunchKernelGGL(k_pc_headpos, dim3(nb), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)kind, (const int32_t*)seg,
                     heads);
  // members with a long column: listed in the key array (free once the
  // groups are known), verified by wavefronts
  int32_t* long_list = reinterpret_cast<int32_t*>(P.key);
  fill_i32(P.total, 0, 1, s);
  hipLaunchKernelGGL(k_pc_verify, dim3(nb), dim3(PSL_BLOCK), 0, s, d, P, (const int32_t*)va, (const int32_t*)kind,
                     (const int32_t*)seg, (const int32_t*)heads, long_list, P.total);
  hipLaunchKernelGGL(k_pc_verify_long, dim3(1024), dim3(PSL_BLOCK), 0, s, d, P, (const int32_t*)va,
                     (const int32_t*)seg, (const int32_t*)heads, (const int32_t*)long_list, (const int32_t*)P.total);
  hipLaunchKernelGGL(k_pc_accum, dim3(nb), dim3(PSL_BLOCK), 0, s, d, P, (const int32_t*)va, (const int32_t*)kind);
  ColScratch Q = P;
  hipLaunchKernelGGL(k_pc_count, dim3(nb), dim3(PSL_BLOCK), 0, s, d, Q);
  scan_excl(d.cnt, d.off, d.n, P.total, ws, s);
  hipLaunchKernelGGL(k_pc_emit, dim3(nb), dim3(PSL_BLOCK), 0, s, d, Q, base, round);
  hipLaunchKernelGGL(k_pc_close, dim3(1), dim3(64), 0, s, d, (const int32_t*)P.total);
}

}  // namespace psl
