// sweep.hip -- one propagation round (section 3.1, "Bound tightening" and
// "Length-based load balancing"; section 3.2, "Internal data structures").
//
// Round semantics (Jacobi): every test reads the bounds as they were when the
// round started (bnd); tightenings are combined in bkey with order-free
// atomic max/min on order-mapped int64 keys; the source row of a final bound
// is the lowest row whose candidate equals it (resolved from a candidate list
// after the sweep). Activities are canonical pairwise trees over the row's CSR
// positions, so every lane grouping below gives the same bits.
//
// Rows are binned by CSR length at ingest. One kernel launch sweeps all bins:
//   bin 0: 4-lane groups (16 rows per wavefront), one pass
//   bin 1: 16-lane groups (4 rows per wavefront), one pass
//   bin 2: one wavefront per row, passes of 64 positions
//   bin 3: one 256-lane workgroup per row, passes of 256 positions
//   bin 4: dense rows, 8192-position chunks per workgroup (partials here,
//          combined by k_dense_finish, propagated by k_dense_prop)
#include "psl_kern.h"
#include "sweep.h"

namespace psl {

#define WAVE_MAXP 64      // passes per wavefront row   (bin 2 rows <= 4096)
#define BLOCK_MAXP 256    // passes per workgroup row   (bin 3 rows <= 65536)
#define DENSE_CHUNK 8192  // positions per dense chunk  (power of two)
#define DENSE_MAXCH 2048  // chunks per dense row

struct Elem {
  int j;
  double a, lb, ub, tmin, tmax;
  bool v, act, imin, imax;
};

template <int MODE>
__device__ __forceinline__ void load_elem(const Dev& d, int64_t p, bool v, Elem& e) {
  e.v = v;
  e.j = 0;
  e.a = 0.0;
  e.lb = 0.0;
  e.ub = 0.0;
  if (v) {
    e.j = d.ci[p];
    e.a = d.va[p];
    double2 b = d.bnd[e.j];
    e.lb = b.x;
    e.ub = b.y;
  }
  e.act = v && (e.lb != e.ub);
  if (MODE == MODE_ROUND) {
    if (v) {
      contrib(e.a, e.lb, e.ub, e.tmin, e.imin, e.tmax, e.imax);
    } else {
      e.tmin = e.tmax = 0.0;
      e.imin = e.imax = false;
    }
  } else {
    // compaction: the constant of the removed columns, kept-entry count
    e.imin = e.imax = false;
    e.tmin = (v && !e.act) ? pos0(e.a * e.lb) : 0.0;
    e.tmax = 0.0;
  }
}

struct RowDec {
  uint8_t code;
  bool infeasible, prop, single;
};

__device__ __forceinline__ RowDec decide_row(const Cfg& c, double lhs, double rhs, int L, int nmin, int nmax,
                                             double minact, double maxact) {
  RowDec r{RC_KEEP, false, false, false};
  bool lo_ok = is_inf(lhs) || (nmin == 0 && minact >= lhs - tol_of(c, lhs));
  bool up_ok = is_inf(rhs) || (nmax == 0 && maxact <= rhs + tol_of(c, rhs));
  if (L == 0) {
    if (lo_ok && up_ok) r.code = RC_EMPTY;
    else r.infeasible = true;
    return r;
  }
  if (lo_ok && up_ok) {
    r.code = RC_REDUNDANT;
    return r;
  }
  if ((nmin == 0 && !is_inf(rhs) && minact > rhs + tol_of(c, rhs)) ||
      (nmax == 0 && !is_inf(lhs) && maxact < lhs - tol_of(c, lhs)))
    r.infeasible = true;
  r.prop = true;
  r.single = (L == 1);
  return r;
}

// Implied bounds of one active entry from the residual activity (the row's
// activity with the entry's own contribution taken out). Side 0 uses rhs and
// the residual min, side 1 lhs and the residual max; a > 0 turns side 0 into an
// upper bound, a < 0 into a lower bound. cap = false when the entry (in a row
// with one active column) yields a side that is not turned into a bound.
__device__ __forceinline__ void prop_elem(const Cfg& c, bool on, const Elem& e, double lhs, double rhs,
                                          double minact, double maxact, int nmin, int nmax, bool single,
                                          bool& cap, bool& hlo, double& tlo, bool& hup, double& tup) {
  cap = true;
  hlo = hup = false;
  tlo = tup = 0.0;
  if (!on) return;
  if (fabs(e.a) < c.coef_tol) {
    cap = false;
    return;
  }
  bool hmin = false, hmax = false;
  double rmin = 0.0, rmax = 0.0;
  if (nmin == 0) {
    rmin = minact - e.tmin;
    hmin = true;
  } else if (nmin == 1 && e.imin) {
    rmin = minact;
    hmin = true;
  }
  if (nmax == 0) {
    rmax = maxact - e.tmax;
    hmax = true;
  } else if (nmax == 1 && e.imax) {
    rmax = maxact;
    hmax = true;
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    double b = side == 0 ? rhs : lhs;
    bool have = side == 0 ? hmin : hmax;
    if (is_inf(b)) continue;
    if (!have) {
      cap = false;
      continue;
    }
    double t = pos0((b - (side == 0 ? rmin : rmax)) / e.a);
    if (!(fabs(t) < c.inf_value)) {
      cap = false;
      continue;
    }
    bool upper = (side == 0) == (e.a > 0);
    if (upper) {
      double u = e.ub;
      bool q = is_inf(u) ? true : (single ? t < u : t < u - c.min_improve * mx1(u));
      if (q) {
        hup = true;
        tup = t;
      }
    } else {
      double l = e.lb;
      bool q = is_inf(l) ? true : (single ? t > l : t > l + c.min_improve * mx1(l));
      if (q) {
        hlo = true;
        tlo = t;
      }
    }
  }
}

// Fold qualifying candidates into the round's accumulators. A candidate that
// is not better than the value read is not the final one unless equal, so
// only candidates <= (>=) the current value go to the source list.
// Must be reached by every lane of the wavefront.
__device__ __forceinline__ void commit_cands(const Dev& d, int row, int j, bool hlo, double tlo, bool hup,
                                             double tup) {
  bool alo = false, aup = false;
  if (hlo) {
    long long* k = &d.bkey[2 * (int64_t)j];
    double cur = dunkey(__atomic_load_n(k, __ATOMIC_RELAXED));
    if (tlo >= cur) {
      alo = true;
      if (tlo > cur) atomicMax(k, dkey(tlo));
    }
  }
  if (hup) {
    long long* k = &d.bkey[2 * (int64_t)j + 1];
    double cur = dunkey(__atomic_load_n(k, __ATOMIC_RELAXED));
    if (tup <= cur) {
      aup = true;
      if (tup < cur) atomicMin(k, dkey(tup));
    }
  }
  wave_append(alo, Cand{2 * j, row, tlo}, d.cand, &d.flags->cand_count);
  wave_append(aup, Cand{2 * j + 1, row, tup}, d.cand, &d.flags->cand_count);
}

__device__ __forceinline__ RowOut row_out_of(uint8_t code, double minact, double maxact, int nmin, int nmax) {
  RowOut o;
  o.j = -1;
  o.pad = 0;
  if (code == RC_EMPTY) {
    o.v0 = minact;
    o.v1 = 0.0;
  } else {
    o.v0 = nmin ? -__builtin_huge_val() : minact;
    o.v1 = nmax ? __builtin_huge_val() : maxact;
  }
  return o;
}

// ---------------------------------------------------------------------------
// bins 0 and 1: G-lane groups, a row in one pass
// ---------------------------------------------------------------------------
template <int G, int MODE>
__device__ __forceinline__ void sweep_groups(const Dev& d, int bin, int lblock) {
  const int per_block = PSL_BLOCK / G;
  int gid = lblock * per_block + (int)(threadIdx.x / G);
  int count = d.bin_off[bin + 1] - d.bin_off[bin];
  bool vr = gid < count;
  int row = vr ? d.bin_rows[d.bin_off[bin] + gid] : 0;
  int gl = threadIdx.x & (G - 1);
  int64_t s0 = 0;
  int len = 0;
  bool on = false;
  if (vr) {
    s0 = d.rp[row];
    len = d.rp[row + 1] - (int)s0;
    on = d.row_on[row] != 0;
  }
  Elem e;
  load_elem<MODE>(d, s0 + gl, on && gl < len, e);
  double minact = group_sum<G>(e.tmin);
  double maxact = group_sum<G>(e.tmax);
  unsigned long long gm = group_mask<G>();
  int nmin = __popcll(__ballot(e.v && e.imin) & gm);
  int nmax = __popcll(__ballot(e.v && e.imax) & gm);
  int L = __popcll(__ballot(e.act) & gm);
  if (MODE == MODE_COMPACT) {
    if (vr && gl == 0) {
      d.row_out[row].v0 = minact;
      d.row_out[row].j = on ? L : 0;
    }
    return;
  }
  bool live = vr && on;
  double lhs = 0.0, rhs = 0.0;
  if (live) {
    lhs = d.lhs[row];
    rhs = d.rhs[row];
  }
  RowDec dec = decide_row(d.cfg, lhs, rhs, L, nmin, nmax, minact, maxact);
  bool prop = live && dec.prop;
  bool cap, hlo, hup;
  double tlo, tup;
  prop_elem(d.cfg, prop && e.act, e, lhs, rhs, minact, maxact, nmin, nmax, dec.single, cap, hlo, tlo, hup, tup);
  commit_cands(d, row, e.j, hlo, tlo, hup, tup);
  bool captured = (__ballot(prop && e.act && !cap) & gm) == 0;
  uint8_t code = RC_KEEP;
  if (live) {
    code = dec.code;
    if (prop && dec.single && !dec.infeasible && captured) code = RC_SINGLETON;
    if (dec.infeasible && gl == 0) atomicOr(&d.flags->infeasible, 1);
  }
  if (vr && gl == 0) d.row_code[row] = code;
  if (live && gl == 0 && (code == RC_EMPTY || code == RC_REDUNDANT))
    d.row_out[row] = row_out_of(code, minact, maxact, nmin, nmax);
  if (live && code == RC_SINGLETON && e.act) d.row_out[row] = RowOut{e.a, 0.0, e.j, 0};
  if (live && code != RC_KEEP && e.act) atomicSub(&d.col_len[e.j], 1);
}

// ---------------------------------------------------------------------------
// bin 2: one wavefront per row, passes of 64 positions
// ---------------------------------------------------------------------------
template <int MODE>
__device__ __forceinline__ void sweep_wave(const Dev& d, int lblock, double* lds) {
  const int bin = BIN_WAVE;
  int w = threadIdx.x >> 6, lane = lane_id();
  int wid = lblock * (PSL_BLOCK / PSL_WAVE) + w;
  int count = d.bin_off[bin + 1] - d.bin_off[bin];
  if (wid >= count) return;  // whole wavefront
  double* ps = lds + w * 2 * WAVE_MAXP;
  int row = d.bin_rows[d.bin_off[bin] + wid];
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  bool on = d.row_on[row] != 0;
  int np = on ? (len + PSL_WAVE - 1) / PSL_WAVE : 0;
  int nmin = 0, nmax = 0, L = 0;
  for (int p = 0; p < np; ++p) {
    int q = p * PSL_WAVE + lane;
    Elem e;
    load_elem<MODE>(d, s0 + q, q < len, e);
    double a = group_sum<PSL_WAVE>(e.tmin);
    double b = group_sum<PSL_WAVE>(e.tmax);
    if (lane == 0) {
      ps[p] = a;
      ps[WAVE_MAXP + p] = b;
    }
    nmin += __popcll(__ballot(e.v && e.imin));
    nmax += __popcll(__ballot(e.v && e.imax));
    L += __popcll(__ballot(e.act));
  }
  double minact = 0.0, maxact = 0.0;
  if (lane == 0) {
    minact = tree_inplace(ps, np);
    maxact = tree_inplace(ps + WAVE_MAXP, np);
  }
  minact = __shfl(minact, 0, PSL_WAVE);
  maxact = __shfl(maxact, 0, PSL_WAVE);
  if (MODE == MODE_COMPACT) {
    if (lane == 0) {
      d.row_out[row].v0 = minact;
      d.row_out[row].j = on ? L : 0;
    }
    return;
  }
  if (!on) {
    if (lane == 0) d.row_code[row] = RC_KEEP;
    return;
  }
  double lhs = d.lhs[row], rhs = d.rhs[row];
  RowDec dec = decide_row(d.cfg, lhs, rhs, L, nmin, nmax, minact, maxact);
  bool uncap = false, mine = false;
  int aj = 0;
  double aa = 0.0;
  if (dec.prop) {
    for (int p = 0; p < np; ++p) {
      int q = p * PSL_WAVE + lane;
      Elem e;
      load_elem<MODE>(d, s0 + q, q < len, e);
      bool cap, hlo, hup;
      double tlo, tup;
      prop_elem(d.cfg, e.act, e, lhs, rhs, minact, maxact, nmin, nmax, dec.single, cap, hlo, tlo, hup, tup);
      commit_cands(d, row, e.j, hlo, tlo, hup, tup);
      uncap |= __ballot(e.act && !cap) != 0;
      if (e.act) {
        mine = true;
        aj = e.j;
        aa = e.a;
      }
    }
  }
  uint8_t code = dec.code;
  if (dec.prop && dec.single && !dec.infeasible && !uncap) code = RC_SINGLETON;
  if (lane == 0) {
    d.row_code[row] = code;
    if (dec.infeasible) atomicOr(&d.flags->infeasible, 1);
    if (code == RC_EMPTY || code == RC_REDUNDANT) d.row_out[row] = row_out_of(code, minact, maxact, nmin, nmax);
  }
  if (code == RC_SINGLETON && mine) {
    d.row_out[row] = RowOut{aa, 0.0, aj, 0};
    atomicSub(&d.col_len[aj], 1);
  }
  if (code == RC_REDUNDANT) {
    for (int p = 0; p < np; ++p) {
      int q = p * PSL_WAVE + lane;
      if (q < len) {
        int j = d.ci[s0 + q];
        double2 b = d.bnd[j];
        if (b.x != b.y) atomicSub(&d.col_len[j], 1);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// workgroup-wide pass sums (bins 3 and 4)
// ---------------------------------------------------------------------------

// Sum of 256 consecutive positions: wavefront butterflies, then
// (w0 + w1) + (w2 + w3). Returns the pass sums in every thread via LDS.
__device__ __forceinline__ void block_pass_sum(double a, double b, double* wl, double& sa, double& sb) {
  int w = threadIdx.x >> 6;
  a = group_sum<PSL_WAVE>(a);
  b = group_sum<PSL_WAVE>(b);
  if (lane_id() == 0) {
    wl[w] = a;
    wl[4 + w] = b;
  }
  __syncthreads();
  sa = (wl[0] + wl[1]) + (wl[2] + wl[3]);
  sb = (wl[4] + wl[5]) + (wl[6] + wl[7]);
  __syncthreads();
}

__device__ __forceinline__ int block_count(bool pred, int* il) {
  int c = __popcll(__ballot(pred));
  int w = threadIdx.x >> 6;
  if (lane_id() == 0) il[w] = c;
  __syncthreads();
  int s = il[0] + il[1] + il[2] + il[3];
  __syncthreads();
  return s;
}

// stats over positions [first, first + 256*np) of the row, pass by pass
template <int MODE>
__device__ __forceinline__ void block_stats(const Dev& d, int64_t s0, int len, int first, int np, double* ps,
                                            int psmax, double* wl, int* il, double& minact, double& maxact,
                                            int& nmin, int& nmax, int& L) {
  nmin = nmax = L = 0;
  for (int p = 0; p < np; ++p) {
    int q = first + p * PSL_BLOCK + (int)threadIdx.x;
    Elem e;
    load_elem<MODE>(d, s0 + q, q < len, e);
    double sa, sb;
    block_pass_sum(e.tmin, e.tmax, wl, sa, sb);
    if (threadIdx.x == 0) {
      ps[p] = sa;
      ps[psmax + p] = sb;
    }
    nmin += block_count(e.v && e.imin, il);
    nmax += block_count(e.v && e.imax, il);
    L += block_count(e.act, il);
  }
  if (threadIdx.x == 0) {
    wl[0] = tree_inplace(ps, np);
    wl[1] = tree_inplace(ps + psmax, np);
  }
  __syncthreads();
  minact = wl[0];
  maxact = wl[1];
  __syncthreads();
}

// propagation / removal bookkeeping over positions [first, first+256*np)
template <int MODE>
__device__ __forceinline__ void block_apply(const Dev& d, int row, int64_t s0, int len, int first, int np,
                                            const RowDec& dec, double lhs, double rhs, double minact,
                                            double maxact, int nmin, int nmax, bool& uncap_any, bool& mine,
                                            int& aj, double& aa, int* il) {
  uncap_any = false;
  mine = false;
  aj = 0;
  aa = 0.0;
  if (dec.prop) {
    bool unc = false;
    for (int p = 0; p < np; ++p) {
      int q = first + p * PSL_BLOCK + (int)threadIdx.x;
      Elem e;
      load_elem<MODE>(d, s0 + q, q < len, e);
      bool cap, hlo, hup;
      double tlo, tup;
      prop_elem(d.cfg, e.act, e, lhs, rhs, minact, maxact, nmin, nmax, dec.single, cap, hlo, tlo, hup, tup);
      commit_cands(d, row, e.j, hlo, tlo, hup, tup);
      unc |= e.act && !cap;
      if (e.act) {
        mine = true;
        aj = e.j;
        aa = e.a;
      }
    }
    uncap_any = block_count(unc, il) > 0;
  } else if (dec.code == RC_REDUNDANT) {
    for (int p = 0; p < np; ++p) {
      int q = first + p * PSL_BLOCK + (int)threadIdx.x;
      if (q < len) {
        int j = d.ci[s0 + q];
        double2 b = d.bnd[j];
        if (b.x != b.y) atomicSub(&d.col_len[j], 1);
      }
    }
  }
}

// bin 3: one workgroup per row
template <int MODE>
__device__ __forceinline__ void sweep_block(const Dev& d, int lblock, double* lds) {
  const int bin = BIN_BLOCK;
  double* ps = lds;
  double* wl = lds + 2 * BLOCK_MAXP;
  int* il = (int*)(wl + 8);
  int row = d.bin_rows[d.bin_off[bin] + lblock];
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  bool on = d.row_on[row] != 0;
  int np = on ? (len + PSL_BLOCK - 1) / PSL_BLOCK : 0;
  double minact, maxact;
  int nmin, nmax, L;
  block_stats<MODE>(d, s0, len, 0, np, ps, BLOCK_MAXP, wl, il, minact, maxact, nmin, nmax, L);
  if (MODE == MODE_COMPACT) {
    if (threadIdx.x == 0) {
      d.row_out[row].v0 = minact;
      d.row_out[row].j = on ? L : 0;
    }
    return;
  }
  if (!on) {
    if (threadIdx.x == 0) d.row_code[row] = RC_KEEP;
    return;
  }
  double lhs = d.lhs[row], rhs = d.rhs[row];
  RowDec dec = decide_row(d.cfg, lhs, rhs, L, nmin, nmax, minact, maxact);
  bool uncap, mine;
  int aj;
  double aa;
  block_apply<MODE>(d, row, s0, len, 0, np, dec, lhs, rhs, minact, maxact, nmin, nmax, uncap, mine, aj, aa, il);
  uint8_t code = dec.code;
  if (dec.prop && dec.single && !dec.infeasible && !uncap) code = RC_SINGLETON;
  if (threadIdx.x == 0) {
    d.row_code[row] = code;
    if (dec.infeasible) atomicOr(&d.flags->infeasible, 1);
    if (code == RC_EMPTY || code == RC_REDUNDANT) d.row_out[row] = row_out_of(code, minact, maxact, nmin, nmax);
  }
  if (code == RC_SINGLETON && mine) {
    d.row_out[row] = RowOut{aa, 0.0, aj, 0};
    atomicSub(&d.col_len[aj], 1);
  }
}

// bin 4 (first launch): partial statistics of one dense chunk
template <int MODE>
__device__ __forceinline__ void sweep_dense_part(const Dev& d, int chunk, double* lds) {
  double* ps = lds;
  const int cmax = DENSE_CHUNK / PSL_BLOCK;
  double* wl = lds + 2 * cmax;
  int* il = (int*)(wl + 8);
  DenseChunk ch = d.dchunk[chunk];
  int row = ch.row;
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  bool on = d.row_on[row] != 0;
  int rem = len - ch.first;
  int np = on ? min(cmax, (rem + PSL_BLOCK - 1) / PSL_BLOCK) : 0;
  double smin, smax;
  int nmin, nmax, L;
  block_stats<MODE>(d, s0, len, ch.first, np, ps, cmax, wl, il, smin, smax, nmin, nmax, L);
  if (threadIdx.x == 0) {
    DensePart pt;
    pt.smin = smin;
    pt.smax = smax;
    pt.nmin = nmin;
    pt.nmax = nmax;
    pt.L = L;
    pt.pad = 0;
    d.dpart[chunk] = pt;
  }
}

template <int MODE>
__global__ void __launch_bounds__(PSL_BLOCK) k_sweep(Dev d, SweepGrid g) {
  __shared__ double lds[2 * BLOCK_MAXP + 16];
  int b = blockIdx.x;
  if (b < g.nb[0]) {
    sweep_groups<4, MODE>(d, BIN_G4, b);
    return;
  }
  b -= g.nb[0];
  if (b < g.nb[1]) {
    sweep_groups<16, MODE>(d, BIN_G16, b);
    return;
  }
  b -= g.nb[1];
  if (b < g.nb[2]) {
    sweep_wave<MODE>(d, b, lds);
    return;
  }
  b -= g.nb[2];
  if (b < g.nb[3]) {
    sweep_block<MODE>(d, b, lds);
    return;
  }
  b -= g.nb[3];
  if (b < g.nb[4]) sweep_dense_part<MODE>(d, b, lds);
}

// combine the chunk partials of each dense row in tree order, then decide
template <int MODE>
__global__ void __launch_bounds__(PSL_BLOCK) k_dense_finish(Dev d) {
  __shared__ double ps[2 * DENSE_MAXCH];
  __shared__ int cnt[3];
  DenseRow& dr = d.drow[blockIdx.x];
  int row = dr.row;
  int nch = dr.nchunk;
  if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
  __syncthreads();
  int a = 0, b = 0, l = 0;
  for (int k = threadIdx.x; k < nch; k += PSL_BLOCK) {
    DensePart pt = d.dpart[dr.chunk0 + k];
    ps[k] = pt.smin;
    ps[DENSE_MAXCH + k] = pt.smax;
    a += pt.nmin;
    b += pt.nmax;
    l += pt.L;
  }
  atomicAdd(&cnt[0], a);
  atomicAdd(&cnt[1], b);
  atomicAdd(&cnt[2], l);
  __syncthreads();
  if (threadIdx.x != 0) return;
  // chunk offsets of kept entries (used by compaction's gather)
  if (MODE == MODE_COMPACT) {
    int run = 0;
    for (int k = 0; k < nch; ++k) {
      int lk = d.dpart[dr.chunk0 + k].L;
      d.dpart[dr.chunk0 + k].pad = run;
      run += lk;
    }
  }
  bool on = d.row_on[row] != 0;
  double minact = tree_inplace(ps, nch);
  double maxact = tree_inplace(ps + DENSE_MAXCH, nch);
  int nmin = cnt[0], nmax = cnt[1], L = cnt[2];
  if (MODE == MODE_COMPACT) {
    d.row_out[row].v0 = minact;
    d.row_out[row].j = on ? L : 0;
    return;
  }
  dr.minact = minact;
  dr.maxact = maxact;
  dr.nmin = nmin;
  dr.nmax = nmax;
  dr.L = L;
  if (!on) {
    dr.keep = 0;
    d.row_code[row] = RC_KEEP;
    return;
  }
  RowDec dec = decide_row(d.cfg, d.lhs[row], d.rhs[row], L, nmin, nmax, minact, maxact);
  dr.keep = dec.code == RC_KEEP ? (dec.infeasible ? 3 : 1) : (dec.code == RC_REDUNDANT ? 2 : 0);
  d.row_code[row] = dec.code;
  if (dec.infeasible) atomicOr(&d.flags->infeasible, 1);
  if (dec.code == RC_EMPTY || dec.code == RC_REDUNDANT)
    d.row_out[row] = row_out_of(dec.code, minact, maxact, nmin, nmax);
}

// propagation (or removal bookkeeping) over one dense chunk
__global__ void __launch_bounds__(PSL_BLOCK) k_dense_prop(Dev d) {
  __shared__ int il[4];
  DenseChunk ch = d.dchunk[blockIdx.x];
  const DenseRow& dr = d.drow[ch.drow];
  if (!d.row_on[ch.row]) return;
  int row = ch.row;
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  int rem = len - ch.first;
  int np = min(DENSE_CHUNK / PSL_BLOCK, (rem + PSL_BLOCK - 1) / PSL_BLOCK);
  RowDec dec;
  dec.code = dr.keep == 2 ? RC_REDUNDANT : (dr.keep == 0 ? RC_EMPTY : RC_KEEP);
  dec.infeasible = dr.keep == 3;
  dec.prop = dr.keep == 1 || dr.keep == 3;
  dec.single = dr.L == 1;
  double lhs = d.lhs[row], rhs = d.rhs[row];
  bool uncap, mine;
  int aj;
  double aa;
  block_apply<MODE_ROUND>(d, row, s0, len, ch.first, np, dec, lhs, rhs, dr.minact, dr.maxact, dr.nmin, dr.nmax,
                          uncap, mine, aj, aa, il);
  // a dense row with one active column: the chunk holding it decides
  if (dec.prop && dec.single && !dec.infeasible && mine) {
    bool cap, hlo, hup;
    double tlo, tup;
    Elem e;
    e.a = aa;
    e.j = aj;
    double2 bb = d.bnd[aj];
    e.lb = bb.x;
    e.ub = bb.y;
    e.v = e.act = true;
    contrib(e.a, e.lb, e.ub, e.tmin, e.imin, e.tmax, e.imax);
    prop_elem(d.cfg, true, e, lhs, rhs, dr.minact, dr.maxact, dr.nmin, dr.nmax, true, cap, hlo, tlo, hup, tup);
    if (cap) {
      d.row_code[row] = RC_SINGLETON;
      d.row_out[row] = RowOut{aa, 0.0, aj, 0};
      atomicSub(&d.col_len[aj], 1);
    }
  }
}

// ---------------------------------------------------------------------------
// source rows of the final bounds
// ---------------------------------------------------------------------------
__global__ void k_src(Dev d) {
  int n = d.flags->cand_count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    Cand c = d.cand[i];
    if (c.t == dunkey(d.bkey[c.js])) atomicMin(&d.src[c.js], c.row);
  }
}

// ---------------------------------------------------------------------------
// decisions per column, record counts per row and column
// ---------------------------------------------------------------------------
__device__ __forceinline__ double empty_value(double c, double lo, double up) {
  if (c > 0) return lo;
  if (c < 0) return up;
  return lo > 0 ? lo : (up < 0 ? up : 0.0);
}

__global__ void k_count(Dev d) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) d.flags->cand_count = 0;
  int64_t m = d.m, n = d.n;
  if (t < m) {
    d.cnt[t] = d.row_code[t] != RC_KEEP;
    return;
  }
  if (t >= m + n) return;
  int j = (int)(t - m);
  double2 b = d.bnd[j];
  if (b.x == b.y) {
    d.col_code[j] = 0;
    d.cnt[t] = 0;
    return;
  }
  double lo = dunkey(d.bkey[2 * (int64_t)j]);
  double up = dunkey(d.bkey[2 * (int64_t)j + 1]);
  uint8_t code = 0;
  int k = 0;
  if (lo != b.x) {
    code |= CC_LB;
    ++k;
  }
  if (up != b.y) {
    code |= CC_UB;
    ++k;
  }
  bool fin = !is_inf(lo) && !is_inf(up);
  if (fin && lo > up + tol_of(d.cfg, up)) code |= CC_INFEAS;
  if (fin && up - lo <= d.cfg.fix_tol * mx1(lo)) {
    code |= CC_FIX;
    ++k;
  } else if (d.col_len[j] == 0) {
    double v = empty_value(d.c[j], lo, up);
    if (is_inf(v)) {
      code |= CC_UNBOUNDED;
    } else {
      code |= CC_EMPTY;
      ++k;
    }
  }
  d.col_code[j] = code;
  d.cnt[t] = k;
  if (code & CC_INFEAS) atomicOr(&d.flags->infeasible, 1);
  if (code & CC_UNBOUNDED) atomicOr(&d.flags->unbounded, 1);
}

__device__ __forceinline__ double coef_in_row(const Dev& d, int row, int j) {
  if (row < 0 || row >= d.m) return __builtin_nan("");  // never taken: a changed bound has a source row
  int lo = d.rp[row], hi = d.rp[row + 1] - 1;
  if (hi < lo) return __builtin_nan("");
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (d.ci[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return d.va[lo];
}

__device__ __forceinline__ Record mkrec(uint8_t type, uint8_t side, int round, int i, int j, int k, double v0,
                                        double v1, double v2, double v3) {
  Record r;
  r.type = type;
  r.side = side;
  r.round = (uint16_t)round;
  r.i = i;
  r.j = j;
  r.k = k;
  r.v[0] = v0;
  r.v[1] = v1;
  r.v[2] = v2;
  r.v[3] = v3;
  return r;
}

__global__ void k_emit(Dev d, int64_t base, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = d.m, n = d.n;
  if (t < m) {
    uint8_t code = d.row_code[t];
    if (code == RC_KEEP) return;
    int i = (int)t;
    RowOut o = d.row_out[i];
    Record* r = d.rec + base + d.off[t];
    if (code == RC_EMPTY) *r = mkrec(REC_EMPTY_ROW, 0, round, i, -1, -1, o.v0, d.lhs[i], d.rhs[i], 0.0);
    else if (code == RC_REDUNDANT) *r = mkrec(REC_REDUNDANT_ROW, 0, round, i, -1, -1, o.v0, o.v1, d.lhs[i], d.rhs[i]);
    else *r = mkrec(REC_SINGLETON_ROW, 0, round, i, o.j, -1, o.v0, d.lhs[i], d.rhs[i], 0.0);
    d.row_on[i] = 0;
    return;
  }
  if (t >= m + n) return;
  int j = (int)(t - m);
  uint8_t code = d.col_code[j];
  if (code == 0) return;
  double2 b = d.bnd[j];
  double lo = dunkey(d.bkey[2 * (int64_t)j]);
  double up = dunkey(d.bkey[2 * (int64_t)j + 1]);
  Record* r = d.rec + base + d.off[t];
  if (code & CC_LB) {
    int s = d.src[2 * (int64_t)j];
    *r++ = mkrec(REC_BOUND_CHANGE, 0, round, -1, j, s, b.x, lo, coef_in_row(d, s, j), 0.0);
  }
  if (code & CC_UB) {
    int s = d.src[2 * (int64_t)j + 1];
    *r++ = mkrec(REC_BOUND_CHANGE, 1, round, -1, j, s, b.y, up, coef_in_row(d, s, j), 0.0);
  }
  double nlo = lo, nup = up;
  if (code & CC_FIX) {
    *r++ = mkrec(REC_FIX_COL, 0, round, -1, j, -1, lo, d.c[j], 0.0, 0.0);
    nlo = nup = lo;
  } else if (code & CC_EMPTY) {
    double v = empty_value(d.c[j], lo, up);
    *r++ = mkrec(REC_EMPTY_COL, 0, round, -1, j, -1, v, d.c[j], 0.0, 0.0);
    nlo = nup = v;
  }
  d.bnd[j] = make_double2(nlo, nup);
  d.bkey[2 * (int64_t)j] = dkey(nlo);
  d.bkey[2 * (int64_t)j + 1] = dkey(nup);
  d.src[2 * (int64_t)j] = 0x7FFFFFFF;
  d.src[2 * (int64_t)j + 1] = 0x7FFFFFFF;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_sweep(const Dev& d, const SweepGrid& g, int mode, hipStream_t s) {
  int total = g.nb[0] + g.nb[1] + g.nb[2] + g.nb[3] + g.nb[4];
  if (total > 0) {
    if (mode == MODE_ROUND) hipLaunchKernelGGL(k_sweep<MODE_ROUND>, dim3(total), dim3(PSL_BLOCK), 0, s, d, g);
    else hipLaunchKernelGGL(k_sweep<MODE_COMPACT>, dim3(total), dim3(PSL_BLOCK), 0, s, d, g);
  }
}

void launch_dense(const Dev& d, int mode, hipStream_t s) {
  if (d.ndense == 0) return;
  if (mode == MODE_ROUND) {
    hipLaunchKernelGGL(k_dense_finish<MODE_ROUND>, dim3(d.ndense), dim3(PSL_BLOCK), 0, s, d);
    hipLaunchKernelGGL(k_dense_prop, dim3(d.nchunks), dim3(PSL_BLOCK), 0, s, d);
  } else {
    hipLaunchKernelGGL(k_dense_finish<MODE_COMPACT>, dim3(d.ndense), dim3(PSL_BLOCK), 0, s, d);
  }
}

void launch_src(const Dev& d, hipStream_t s) { hipLaunchKernelGGL(k_src, dim3(1024), dim3(PSL_BLOCK), 0, s, d); }

void launch_count(const Dev& d, hipStream_t s) {
  int64_t t = (int64_t)d.m + d.n;
  unsigned blocks = (unsigned)((t + PSL_BLOCK - 1) / PSL_BLOCK);
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_count, dim3(blocks), dim3(PSL_BLOCK), 0, s, d);
}

void launch_emit(const Dev& d, int64_t base, int round, hipStream_t s) {
  int64_t t = (int64_t)d.m + d.n;
  if (t == 0) return;
  unsigned blocks = (unsigned)((t + PSL_BLOCK - 1) / PSL_BLOCK);
  hipLaunchKernelGGL(k_emit, dim3(blocks), dim3(PSL_BLOCK), 0, s, d, base, round);
}

int dense_chunk_size() { return DENSE_CHUNK; }
int dense_max_chunks() { return DENSE_MAXCH; }
int wave_max_len() { return WAVE_MAXP * PSL_WAVE; }
int block_max_len() { return BLOCK_MAXP * PSL_BLOCK; }

}  // namespace psl
