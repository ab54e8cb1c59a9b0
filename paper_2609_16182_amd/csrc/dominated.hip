// dominated.hip -- dominated columns through implied dual bounds (a dual
// explorer, section 2.1: it keeps at least one optimal solution), once per
// outer cycle after the parallel columns.
//
// Row duals (c - A'y - z = 0) are bounded by the rows' sides (only a finite
// lhs: y >= 0; only a finite rhs: y <= 0) and by column singletons (a column
// in one alive row with coefficient a, |a| >= coef_tol: no upper bound gives
// z >= 0, a y <= c; no lower bound z <= 0, a y >= c), kept as order-mapped
// keys so that the singletons' bounds meet by atomic max / min. Then every
// active column in an alive row gets the range of its reduced cost,
// [c - sum max(a y), c - sum min(a y)], each sum the canonical pairwise tree
// over the column's stored positions of the transposed copy (dead rows and
// +0 entries give +0; an infinite term makes that end infinite): 16-lane
// groups for columns of at most 16 positions (the group's butterfly is the
// tree), a wavefront per longer column (one position per lane up to 64, else
// aligned blocks of positions per lane, each summed as its own subtree, then
// the butterfly). A lower end above feas_tol max(1, |c|) fixes the column at
// its lower bound, an upper end below the negative tolerance at its upper
// bound (an infinite one: unbounded or infeasible); crossing bounds of a row
// (beyond the tolerance) also mean unbounded or infeasible, a smaller
// crossing skips the LP's pass. DOMINATED_COL records in column order.
#include "psl_kern.h"
#include "sweep.h"

namespace psl {

#define DOM_SHORT 16
#define DOM_SKIP 1
#define DOM_UNBOUNDED 2

__device__ __forceinline__ bool dom_lp_stopped(const Dev& d, int lp) {
  if (d.K > 1) return d.lp_ok[lp] == 0;
  return (d.flags->infeasible | d.flags->unbounded) != 0;
}

__global__ void k_dom_rows(Dev d, DomScratch S) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += stride) {
    double lo = 0.0, hi = 0.0;
    if (d.row_on[i]) {
      bool lf = !is_inf(d.lhs[i]), rf = !is_inf(d.rhs[i]);
      if (lf || rf) {
        lo = lf && !rf ? 0.0 : -__builtin_inf();
        hi = rf && !lf ? 0.0 : __builtin_inf();
      }
    }
    S.ykey[2 * i] = dkey(lo);
    S.ykey[2 * i + 1] = dkey(hi);
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < d.K; k += stride) S.lp_flag[k] = 0;
}

// the bounds a column singleton puts on its row's dual
__global__ void k_dom_singletons(Dev d, DomScratch S) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.n) return;
  int j = (int)t;
  double2 b = d.bnd[j];
  if (b.x == b.y || d.col_len[j] != 1 || dom_lp_stopped(d, col_lp_of(d, j))) return;
  if (!is_inf(b.x) && !is_inf(b.y)) return;
  int i = -1;
  double a = 0.0;
  for (int q = d.cp[j]; q < d.cp[j + 1]; ++q)
    if (d.row_on[d.ri[q]]) {
      i = d.ri[q];
      a = d.cva[q];
      break;
    }
  if (i < 0 || fabs(a) < d.cfg.coef_tol) return;
  long long v = dkey(pos0(d.c[j] / a));
  if (is_inf(b.y)) {
    if (a > 0) atomicMin(&S.ykey[2 * (int64_t)i + 1], v);
    else atomicMax(&S.ykey[2 * (int64_t)i], v);
  }
  if (is_inf(b.x)) {
    if (a > 0) atomicMax(&S.ykey[2 * (int64_t)i], v);
    else atomicMin(&S.ykey[2 * (int64_t)i + 1], v);
  }
}

// crossing bounds: the LP's pass is skipped, or the LP is unbounded
__global__ void k_dom_cross(Dev d, DomScratch S) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m || !d.row_on[i]) return;
  double lo = dunkey(S.ykey[2 * i]), hi = dunkey(S.ykey[2 * i + 1]);
  if (lo > hi) atomicOr(&S.lp_flag[row_lp_of(d, (int)i)], lo > hi + tol_of(d.cfg, hi) ? DOM_UNBOUNDED : DOM_SKIP);
}

// terms of position q of a column (max and min of a y over the row's bounds)
__device__ __forceinline__ void dom_terms(const Dev& d, const DomScratch& S, int q, bool in, double& th, double& tl,
                                          int& ih, int& il) {
  th = tl = 0.0;
  ih = il = 0;
  if (!in) return;
  int i = d.ri[q];
  double a = d.cva[q];
  if (!d.row_on[i] || a == 0.0) return;
  double lo = dunkey(S.ykey[2 * (int64_t)i]), hi = dunkey(S.ykey[2 * (int64_t)i + 1]);
  double mx = a > 0 ? a * hi : a * lo;
  double mn = a > 0 ? a * lo : a * hi;
  if (is_inf(mx)) ih = 1;
  else th = pos0(mx);
  if (is_inf(mn)) il = 1;
  else tl = pos0(mn);
}

// the decision from the two sums: 0 lower bound, 1 upper bound, -1 none
__device__ __forceinline__ int dom_side(const Dev& d, int k, double sh, double sl, int ih, int il) {
  double ck = d.c[k], tol = tol_of(d.cfg, ck);
  if (ih == 0 && ck - sh > tol) return 0;
  if (il == 0 && ck - sl < -tol) return 1;
  return -1;
}

__device__ __forceinline__ bool dom_candidate(const Dev& d, const DomScratch& S, int k) {
  double2 b = d.bnd[k];
  int lp = col_lp_of(d, k);
  return b.x != b.y && d.col_len[k] >= 1 && !dom_lp_stopped(d, lp) && S.lp_flag[lp] == 0;
}

// 16-lane groups, columns of at most DOM_SHORT positions; longer candidates
// go to the list (n_long counts them)
__global__ void __launch_bounds__(PSL_BLOCK) k_dom_short(Dev d, DomScratch S, int32_t* long_list, int32_t* n_long) {
  int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / DOM_SHORT;
  int gl = threadIdx.x & (DOM_SHORT - 1);
  bool vk = g < d.n;
  int k = vk ? (int)g : 0;
  bool cand = vk && dom_candidate(d, S, k);
  int q0 = cand ? d.cp[k] : 0, len = cand ? d.cp[k + 1] - q0 : 0;
  if (cand && len > DOM_SHORT) {
    if (gl == 0) long_list[atomicAdd(n_long, 1)] = k;
    cand = false;
    len = 0;
  }
  double th, tl;
  int ih, il;
  dom_terms(d, S, q0 + gl, cand && gl < len, th, tl, ih, il);
  double sh = group_sum<DOM_SHORT>(th), sl = group_sum<DOM_SHORT>(tl);
  ih = (int)group_sum_u64<DOM_SHORT>((unsigned long long)ih);
  il = (int)group_sum_u64<DOM_SHORT>((unsigned long long)il);
  if (vk && gl == 0) S.side[k] = cand ? (int8_t)dom_side(d, k, sh, sl, ih, il) : (int8_t)-1;
}

// a lane's aligned block [b0, b0 + c) of a column's positions (c a power of
// two), summed as its own pairwise subtree with a stack of partial sums
__device__ __forceinline__ void dom_block(const Dev& d, const DomScratch& S, int q0, int len, int b0, int c,
                                          double& sh, double& sl, int& ih, int& il) {
  double st_h[32], st_l[32];
  int top = 0;
  ih = il = 0;
  for (int t = 0; t < c; ++t) {
    double th, tl;
    int a, b;
    dom_terms(d, S, q0 + b0 + t, b0 + t < len, th, tl, a, b);
    ih += a;
    il += b;
    // merge while the stack's top block has the size of the new one
    for (int w = t; w & 1; w >>= 1) {
      --top;
      th = st_h[top] + th;
      tl = st_l[top] + tl;
    }
    st_h[top] = th;
    st_l[top] = tl;
    ++top;
  }
  sh = st_h[0];
  sl = st_l[0];
}

// a wavefront per listed column
__global__ void __launch_bounds__(PSL_BLOCK) k_dom_long(Dev d, DomScratch S, const int32_t* long_list,
                                                         const int32_t* n_long) {
  int nl = *n_long;
  int lane = lane_id();
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int w = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); w < nl; w += wstride) {
    int k = long_list[w];
    int q0 = d.cp[k], len = d.cp[k + 1] - q0;
    int p = PSL_WAVE;
    while (p < len) p <<= 1;
    int c = p / PSL_WAVE;
    double sh, sl;
    int ih, il;
    dom_block(d, S, q0, len, lane * c, c, sh, sl, ih, il);
    sh = group_sum<PSL_WAVE>(sh);
    sl = group_sum<PSL_WAVE>(sl);
    ih = (int)group_sum_u64<PSL_WAVE>((unsigned long long)ih);
    il = (int)group_sum_u64<PSL_WAVE>((unsigned long long)il);
    if (lane == 0) S.side[k] = (int8_t)dom_side(d, k, sh, sl, ih, il);
  }
}

__global__ void k_dom_count(Dev d, DomScratch S) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  int sd = S.side[j];
  int c = 0;
  if (sd >= 0) {
    double2 b = d.bnd[j];
    double v = sd == 0 ? b.x : b.y;
    if (is_inf(v)) flag_unbounded(d, col_lp_of(d, (int)j));
    else c = 1;
  }
  d.cnt[j] = c;
}

__global__ void k_dom_emit(Dev d, DomScratch S, int64_t base, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.n) return;
  int sd = S.side[t];
  if (sd < 0) return;
  int j = (int)t;
  double2 b = d.bnd[j];
  double v = sd == 0 ? b.x : b.y;
  if (is_inf(v)) return;
  int lp = col_lp_of(d, j);
  Record r;
  r.type = REC_DOMINATED_COL;
  r.side = (uint8_t)sd;
  r.round = (uint16_t)round_of(d, lp, round);
  r.i = -1;
  r.j = j;
  r.k = -1;
  r.v[0] = v;
  r.v[1] = d.c[j];
  r.v[2] = 0.0;
  r.v[3] = 0.0;
  d.rec[base + d.flags->round_total + d.off[t]] = r;
  d.bnd[j] = make_double2(v, v);
  d.bkey[2 * (int64_t)j] = dkey(v);
  d.bkey[2 * (int64_t)j + 1] = dkey(v);
  d.flags->merged = 1;
  if (d.K > 1) d.lpf[lp].merged = 1;
}

// LPs whose dual bounds crossed beyond the tolerance are unbounded or infeasible
__global__ void k_dom_close(Dev d, DomScratch S) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < d.K && (S.lp_flag[k] & DOM_UNBOUNDED)) flag_unbounded(d, (int)k);
  if (k == 0) d.flags->round_total += *S.total;
}

void launch_dominated(const Dev& d, const DomScratch& S, int64_t base, int round, int32_t* ws, hipStream_t s) {
  unsigned mb = (unsigned)((d.m + PSL_BLOCK - 1) / PSL_BLOCK);
  unsigned kb = (unsigned)((d.K + PSL_BLOCK - 1) / PSL_BLOCK);
  unsigned rb = mb > kb ? mb : kb;
  if (rb > 8192) rb = 8192;
  if (rb < 1) rb = 1;
  hipLaunchKernelGGL(k_dom_rows, dim3(rb), dim3(PSL_BLOCK), 0, s, d, S);
  if (d.n == 0) {
    fill_i32(S.total, 0, 1, s);
  } else {
    unsigned nb = (unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK);
    hipLaunchKernelGGL(k_dom_singletons, dim3(nb), dim3(PSL_BLOCK), 0, s, d, S);
    if (d.m > 0) hipLaunchKernelGGL(k_dom_cross, dim3(mb), dim3(PSL_BLOCK), 0, s, d, S);
    // the long columns' list in d.cnt (free until the count pass), its length
    // in S.total
    fill_i32(S.total, 0, 1, s);
    int64_t gb = ((int64_t)d.n * DOM_SHORT + PSL_BLOCK - 1) / PSL_BLOCK;
    hipLaunchKernelGGL(k_dom_short, dim3((unsigned)gb), dim3(PSL_BLOCK), 0, s, d, S, d.cnt, S.total);
    hipLaunchKernelGGL(k_dom_long, dim3(1024), dim3(PSL_BLOCK), 0, s, d, S, (const int32_t*)d.cnt,
                       (const int32_t*)S.total);
    hipLaunchKernelGGL(k_dom_count, dim3(nb), dim3(PSL_BLOCK), 0, s, d, S);
    scan_excl(d.cnt, d.off, d.n, S.total, ws, s);
    hipLaunchKernelGGL(k_dom_emit, dim3(nb), dim3(PSL_BLOCK), 0, s, d, S, base, round);
  }
  hipLaunchKernelGGL(k_dom_close, dim3(kb > 0 ? kb : 1), dim3(PSL_BLOCK), 0, s, d, S);
}

}  // namespace psl
