// sweep.hip -- one propagation round (section 3.1, "Bound tightening" and
// "Length-based load balancing"; section 3.2, "Internal data structures").
//
// Round semantics (Jacobi): every test reads the bounds as they were when the
// round started (bnd); tightenings are combined in bkey with order-free
// atomic max/min on order-mapped int64 keys; the source row of a final bound
// is the lowest row whose candidate equals it (resolved from a candidate list
// after the sweep). Activities are canonical pairwise trees over the row's CSR
// positions (leaves padded with +0 to a power of two), so every aligned
// power-of-two grouping of positions -- C contiguous positions per lane, a
// butterfly over G lanes, four wavefronts, chunk partials -- gives the same
// bits, whatever bin a row falls in.
//
// Bins (by CSR length; rows are listed per bin, ascending):
//   G4  <= 4     4-lane groups, 1 position per lane
//   G16 <= 16    16-lane groups, 1 position per lane
//   W1  <= 64    one wavefront, 1 position per lane
//   W4  <= 256   one wavefront, 4 contiguous positions per lane
//   W8  <= 512   one wavefront, 8 contiguous positions per lane
//   LONG         chunks of npass * 2048 positions, one workgroup each:
//                k_long_stats writes chunk partials, then k_sweep combines
//                them in tree order and propagates chunk by chunk.
// Each row is handled in one pass with its elements kept in registers.
#include "psl_kern.h"
#include "sweep.h"

namespace psl {


struct El {
  int j;
  double a, lb, ub;
  bool v;
};

// Elements at positions s0 + base + k (k < C) of a row, valid when on and
// base + k < len. All loads are issued before any is used, without branches
// between them (an invalid element reads position 0, which exists whenever
// the matrix has an entry), so a lane has C gathers in flight at once.
template <int C>
__device__ __forceinline__ void load_els(const Dev& d, int64_t s0, int len, int base, bool on, El (&e)[C]) {
  int j[C];
  double a[C];
  double2 b[C];
  bool v[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    v[k] = on && base + k < len;
    j[k] = 0;
    a[k] = 0.0;
    b[k] = make_double2(0.0, 0.0);
  }
  if (d.nnz > 0) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      int64_t p = v[k] ? s0 + base + k : 0;
      j[k] = d.ci[p];
      a[k] = d.va[p];
    }
#pragma unroll
    for (int k = 0; k < C; ++k) b[k] = d.bnd[j[k]];
  }
#pragma unroll
  for (int k = 0; k < C; ++k) {
    e[k].v = v[k];
    e[k].j = v[k] ? j[k] : 0;
    e[k].a = v[k] ? a[k] : 0.0;
    e[k].lb = v[k] ? b[k].x : 0.0;
    e[k].ub = v[k] ? b[k].y : 0.0;
  }
}

__device__ __forceinline__ bool el_active(const El& e) { return e.v && e.lb != e.ub; }

// activity terms of one element and its packed counts
// (bit 0: infinite min contribution, bit 10: infinite max, bit 20: active)
// (straight-line: an invalid element holds a = lb = ub = 0 and so gives +0
// terms and no counts)
template <int MODE>
__device__ __forceinline__ void el_terms(const El& e, double& tmin, double& tmax, int& cnt) {
  tmin = tmax = 0.0;
  cnt = 0;
  bool act = e.v && e.lb != e.ub;
  if (MODE == MODE_ROUND) {
    bool imin, imax;
    contrib(e.a, e.lb, e.ub, tmin, imin, tmax, imax);
    cnt = (imin ? 1 : 0) | (imax ? 1 << 10 : 0) | (act ? 1 << 20 : 0);
  } else {
    // compaction: constant of the removed columns; active-entry count
    tmin = act ? 0.0 : pos0(e.a * e.lb);
    cnt = act ? 1 << 20 : 0;
  }
}

__device__ __forceinline__ int cnt_min(int c) { return c & 1023; }
__device__ __forceinline__ int cnt_max(int c) { return (c >> 10) & 1023; }
__device__ __forceinline__ int cnt_act(int c) { return c >> 20; }

template <int G>
__device__ __forceinline__ int group_sum_int(int x) {
#pragma unroll
  for (int s = 1; s < G; s <<= 1) x += __shfl_xor(x, s, PSL_WAVE);
  return x;
}

// pairwise tree over C values held in registers (C a power of two)
template <int C>
__device__ __forceinline__ double lane_tree(double (&x)[C]) {
#pragma unroll
  for (int w = 1; w < C; w <<= 1)
#pragma unroll
    for (int i = 0; i < C; i += 2 * w) x[i] = x[i] + x[i + w];
  return x[0];
}

// load C contiguous positions [base, base + C) of a row and reduce them
template <int C, int MODE>
__device__ __forceinline__ void lane_stats(const Dev& d, int64_t s0, int len, int base, El (&e)[C], double& smin,
                                           double& smax, int& cnt) {
  double a[C], b[C];
  cnt = 0;
  load_els<C>(d, s0, len, base, true, e);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    int c;
    el_terms<MODE>(e[k], a[k], b[k], c);
    cnt += c;
  }
  smin = lane_tree<C>(a);
  smax = lane_tree<C>(b);
}

struct RowDec {
  uint8_t code;
  bool infeasible, prop, single;
  int force;  // forcing row: 1 at its min activity (= rhs), 2 at its max (= lhs)
};

// Row decisions from the round's statistics. any_tiny: the row has an active
// entry with |a| < coef_tol (such a row is never forcing: its column could
// move far within the tolerance).
__device__ __forceinline__ RowDec decide_row(const Cfg& c, double lhs, double rhs, int L, int nmin, int nmax,
                                             double minact, double maxact, bool any_tiny) {
  RowDec r{RC_KEEP, false, false, false, 0};
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
  // A side gives an entry a bound only when the residual activity on that side
  // is finite, i.e. with at most one infinite contribution (the entry's own);
  // with none on either side the row yields no candidate and is not re-read.
  // (A row with one active column has at most one infinite contribution per
  // side, so it always propagates on its finite sides.)
  r.prop = (!is_inf(rhs) && nmin <= 1) || (!is_inf(lhs) && nmax <= 1);
  r.single = (L == 1);
  // Forcing rows (at least two active columns): the finite min activity
  // reaching rhs (or the max reaching lhs) within tol leaves every active
  // column at the bound of that contribution; the row leaves and those
  // bounds become candidates.
  if (c.forcing && !r.infeasible && L >= 2 && !any_tiny) {
    if (nmin == 0 && !is_inf(rhs) && minact >= rhs - tol_of(c, rhs)) r.force = 1;
    else if (nmax == 0 && !is_inf(lhs) && maxact <= lhs + tol_of(c, lhs)) r.force = 2;
    if (r.force) r.code = r.force == 1 ? RC_FORCE_MIN : RC_FORCE_MAX;
  }
  return r;
}

__device__ __forceinline__ bool is_forcing(uint8_t code) { return code == RC_FORCE_MIN || code == RC_FORCE_MAX; }

struct RowStat {
  double minact, maxact;
  int nmin, nmax;
};

// Implied bounds of one active entry from the residual activity (the row's
// activity with the entry's own contribution taken out). Side 0 uses rhs and
// the residual min, side 1 lhs and the residual max; a > 0 turns side 0 into an
// upper bound, a < 0 into a lower bound. cap = false when a finite side yields
// no bound (it matters for rows with one active column, which are removed only
// when every finite side became a bound).
__device__ __forceinline__ void prop_el(const Cfg& c, bool on, const El& e, double lhs, double rhs, const RowStat& st,
                                        bool single, int force, bool& cap, bool& hlo, double& tlo, bool& hup,
                                        double& tup) {
  cap = true;
  hlo = hup = false;
  tlo = tup = 0.0;
  if (!on) return;
  if (force) {
    // a forcing row: the column's other bound moves onto the forced one
    // (min side: a > 0 at lb, a < 0 at ub; max side the other way round)
    if ((force == 1) == (e.a > 0)) {
      hup = e.lb < e.ub;
      tup = e.lb;
    } else {
      hlo = e.ub > e.lb;
      tlo = e.ub;
    }
    return;
  }
  if (fabs(e.a) < c.coef_tol) {
    cap = false;
    return;
  }
  double tmin, tmax;
  bool imin, imax;
  contrib(e.a, e.lb, e.ub, tmin, imin, tmax, imax);
  bool hmin = false, hmax = false;
  double rmin = 0.0, rmax = 0.0;
  if (st.nmin == 0) {
    rmin = st.minact - tmin;
    hmin = true;
  } else if (st.nmin == 1 && imin) {
    rmin = st.minact;
    hmin = true;
  }
  if (st.nmax == 0) {
    rmax = st.maxact - tmax;
    hmax = true;
  } else if (st.nmax == 1 && imax) {
    rmax = st.maxact;
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

struct CandSink {  // this workgroup's candidate region and its LDS counter
  Cand* list;
  int32_t* counter;
};

// Fold qualifying candidates into the round's accumulators. A candidate that
// is not better than the value read cannot be the final one unless equal, so
// only candidates <= (>=) the current value go to the source list.
// Must be reached by every lane of the wavefront.
__device__ __forceinline__ void commit_cands(const Dev& d, const CandSink& sk, int pos, int j, bool hlo, double tlo,
                                             bool hup, double tup) {
  bool alo = false, aup = false;
  if (hlo) {
    long long* k = &d.bkey[2 * (int64_t)j];
    double cur = dunkey(*k);  // may be stale (larger): only costs an extra atomic
    if (tlo >= cur) {
      alo = true;
      if (tlo > cur) atomicMax(k, dkey(tlo));
    }
  }
  if (hup) {
    long long* k = &d.bkey[2 * (int64_t)j + 1];
    double cur = dunkey(*k);
    if (tup <= cur) {
      aup = true;
      if (tup < cur) atomicMin(k, dkey(tup));
    }
  }
  wave_append(alo, Cand{2 * j, pos, tlo}, sk.list, sk.counter);
  wave_append(aup, Cand{2 * j + 1, pos, tup}, sk.list, sk.counter);
}

__device__ __forceinline__ RowOut row_out_of(uint8_t code, const RowStat& st) {
  RowOut o;
  o.j = -1;
  o.pad = 0;
  if (code == RC_EMPTY || code == RC_FORCE_MIN) {
    o.v0 = st.minact;
    o.v1 = 0.0;
  } else if (code == RC_FORCE_MAX) {
    o.v0 = st.maxact;
    o.v1 = 0.0;
  } else {
    o.v0 = st.nmin ? -__builtin_huge_val() : st.minact;
    o.v1 = st.nmax ? __builtin_huge_val() : st.maxact;
  }
  return o;
}

// propagate the C register-held elements of a lane; tracks the one active
// element of a row with L == 1 and whether some entry left a side unbounded
template <int C>
__device__ __forceinline__ void lane_prop(const Dev& d, const CandSink& sk, int64_t p0, bool prop, const El (&e)[C],
                                          double lhs, double rhs,
                                          const RowStat& st, bool single, int force, bool& uncap, bool& mine,
                                          int& aj, double& aa) {
#pragma unroll
  for (int k = 0; k < C; ++k) {
    bool act = prop && el_active(e[k]);
    bool cap, hlo, hup;
    double tlo, tup;
    prop_el(d.cfg, act, e[k], lhs, rhs, st, single, force, cap, hlo, tlo, hup, tup);
    commit_cands(d, sk, (int)(p0 + k), e[k].j, hlo, tlo, hup, tup);
    if (act && !cap) uncap = true;
    if (act) {
      mine = true;
      aj = e[k].j;
      aa = e[k].a;
    }
  }
}

// the same, loading the elements again in groups of (at most) four, so that
// wide lanes do not keep C elements live while each group's gathers are in
// flight together
#define STREAM_GROUP 4
template <int C>
__device__ __forceinline__ void lane_prop_stream(const Dev& d, const CandSink& sk, int row, bool prop, int64_t s0,
                                                 int len, int base, double lhs, double rhs, const RowStat& st,
                                                 bool single, int force, bool& uncap, bool& mine, int& aj,
                                                 double& aa) {
  constexpr int GS = C < STREAM_GROUP ? C : STREAM_GROUP;
#pragma unroll 1
  for (int g = 0; g < C; g += GS) {
    El e[GS];
    load_els<GS>(d, s0, len, base + g, prop, e);
#pragma unroll
    for (int k = 0; k < GS; ++k) {
      bool act = el_active(e[k]);
      bool cap, hlo, hup;
      double tlo, tup;
      prop_el(d.cfg, act, e[k], lhs, rhs, st, single, force, cap, hlo, tlo, hup, tup);
      commit_cands(d, sk, (int)(s0 + base + g + k), e[k].j, hlo, tlo, hup, tup);
      if (act && !cap) uncap = true;
      if (act) {
        mine = true;
        aj = e[k].j;
        aa = e[k].a;
      }
    }
  }
}

template <int C>
__device__ __forceinline__ void lane_drop_stream(const Dev& d, bool on, int64_t s0, int len, int base, double lhs,
                                                 double rhs) {
  constexpr int GS = C < STREAM_GROUP ? C : STREAM_GROUP;
#pragma unroll 1
  for (int g = 0; g < C; g += GS) {
    El e[GS];
    load_els<GS>(d, s0, len, base + g, on, e);
#pragma unroll
    for (int k = 0; k < GS; ++k)
      if (el_active(e[k])) drop_col(d, e[k].j, e[k].a, lhs, rhs);
  }
}

template <int C>
__device__ __forceinline__ void lane_drop(const Dev& d, const El (&e)[C], double lhs, double rhs) {
#pragma unroll
  for (int k = 0; k < C; ++k)
    if (el_active(e[k])) drop_col(d, e[k].j, e[k].a, lhs, rhs);
}

// ---------------------------------------------------------------------------
// rows of at most G*C entries: one G-lane group per row, C positions per lane
// ---------------------------------------------------------------------------

// what a lane reads of its row in a row block
template <int C>
struct RowIn {
  bool vr, on;   // the lane's group has a row; the row is active
  int row, len;
  int64_t s0;
  double lhs, rhs;
  El e[C];
};

// First level of a row block's loads: the bin entry of the lane's row. A
// lane without a row reads the bin's first entry (the workgroup exists
// because the bin has one), so no load of the row block is conditional.
template <int G, int C>
__device__ __forceinline__ void row_entry(const Dev& d, int bin, int vblock, RowIn<C>& in) {
  const int per_block = PSL_BLOCK / G;
  int gid = vblock * per_block + (int)(threadIdx.x / G);
  int count = d.bin_off[bin + 1] - d.bin_off[bin];
  in.vr = gid < count;
  BinEnt be = d.bins[d.bin_off[bin] + (in.vr ? gid : 0)];
  in.row = be.row;
  in.s0 = be.start;
  in.len = in.vr ? be.len : 0;
}

// Second level: the row's flag and sides and the lane's positions (columns
// and coefficients); the third level, the bounds, is issued by load_els or
// by the caller.
template <int G, int C>
__device__ __forceinline__ void row_data(const Dev& d, RowIn<C>& in) {
  in.on = in.vr && d.row_on[in.row] != 0;
  in.lhs = d.lhs[in.row];
  in.rhs = d.rhs[in.row];
}

// statistics, decisions, candidates and removals of the row block's rows
// from the loaded inputs (elements of inactive rows are cleared here)
template <int G, int C, int MODE>
__device__ __forceinline__ void row_block(const Dev& d, const CandSink& sk, RowIn<C>& in) {
  const bool vr = in.vr, on = in.on;
  const int row = in.row, len = in.len;
  const int64_t s0 = in.s0;
  int gl = threadIdx.x & (G - 1);
  El(&e)[C] = in.e;
  double smin, smax;
  int cnt = 0;
  {
    double a[C], b[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if (!on) e[k] = El{0, 0.0, 0.0, 0.0, false};
      int c;
      el_terms<MODE>(e[k], a[k], b[k], c);
      cnt += c;
    }
    smin = lane_tree<C>(a);
    smax = lane_tree<C>(b);
  }
  RowStat st;
  st.minact = group_sum<G>(smin);
  st.maxact = group_sum<G>(smax);
  cnt = group_sum_int<G>(cnt);
  st.nmin = cnt_min(cnt);
  st.nmax = cnt_max(cnt);
  int L = cnt_act(cnt);
  if (MODE == MODE_COMPACT) {
    if (vr && gl == 0) {
      d.row_out[row].v0 = st.minact;
      d.row_out[row].j = on ? L : 0;
    }
    return;
  }
  bool live = vr && on;
  double lhs = live ? in.lhs : 0.0, rhs = live ? in.rhs : 0.0;
  if (live && gl == 0) d.rinf[row] = make_int2(st.nmin, st.nmax);
  bool tiny = false;
#pragma unroll
  for (int k = 0; k < C; ++k) tiny = tiny || (el_active(e[k]) && fabs(e[k].a) < d.cfg.coef_tol);
  bool any_tiny = (__ballot(tiny) & group_mask<G>()) != 0;
  RowDec dec = decide_row(d.cfg, lhs, rhs, L, st.nmin, st.nmax, st.minact, st.maxact, any_tiny);
  bool prop = live && dec.prop;
  bool uncap = false, mine = false;
  int aj = 0;
  double aa = 0.0;
  int force = live ? dec.force : 0;
  if (C == 1) lane_prop<C>(d, sk, s0 + gl * C, prop, e, lhs, rhs, st, dec.single, force, uncap, mine, aj, aa);
  else  // reload (L1/L2 hits) instead of keeping C elements live through the sums
    lane_prop_stream<C>(d, sk, row, prop, s0, len, gl * C, lhs, rhs, st, dec.single, force, uncap, mine, aj, aa);
  bool captured = (__ballot(uncap) & group_mask<G>()) == 0;
  uint8_t code = RC_KEEP;
  if (live) {
    code = dec.code;
    if (prop && dec.single && !dec.infeasible && captured) code = RC_SINGLETON;
    if (dec.infeasible && gl == 0) flag_infeasible(d, row_lp_of(d, row));
  }
  if (vr && gl == 0) d.row_code[row] = code;
  if (live && gl == 0 && (code == RC_EMPTY || code == RC_REDUNDANT || is_forcing(code)))
    d.row_out[row] = row_out_of(code, st);
  if (code == RC_SINGLETON && mine) {
    d.row_out[row] = RowOut{aa, 0.0, aj, 0};
    drop_col(d, aj, aa, lhs, rhs);
  }
  if (code == RC_REDUNDANT || is_forcing(code)) {
    if (C == 1) lane_drop<C>(d, e, lhs, rhs);
    else lane_drop_stream<C>(d, live, s0, len, gl * C, lhs, rhs);
  }
}

// The workgroup's REP row blocks of the bin. With one position per lane the
// loads of all REP blocks are issued level by level before any block is
// processed, so a lane has REP rows' gathers in flight together.
template <int G, int C, int MODE, int REP>
__device__ __forceinline__ void sweep_rows(const Dev& d, const CandSink& sk, int bin, int lblock) {
  int count = d.bin_off[bin + 1] - d.bin_off[bin];
  int gl = threadIdx.x & (G - 1);
  if (C == 1) {
    RowIn<C> in[REP];
    int j[REP];
    double a[REP];
#pragma unroll
    for (int k = 0; k < REP; ++k) row_entry<G, C>(d, bin, lblock * REP + k, in[k]);
#pragma unroll
    for (int k = 0; k < REP; ++k) {
      row_data<G, C>(d, in[k]);
      bool v = gl < in[k].len;
      int64_t p = v ? in[k].s0 + gl : 0;
      j[k] = d.ci[p];
      a[k] = d.va[p];
      in[k].e[0].v = v;
    }
#pragma unroll
    for (int k = 0; k < REP; ++k) {
      double2 bb = d.bnd[j[k]];
      bool v = in[k].e[0].v;
      in[k].e[0].j = v ? j[k] : 0;
      in[k].e[0].a = v ? a[k] : 0.0;
      in[k].e[0].lb = v ? bb.x : 0.0;
      in[k].e[0].ub = v ? bb.y : 0.0;
    }
#pragma unroll
    for (int k = 0; k < REP; ++k) {
      if ((lblock * REP + k) * (PSL_BLOCK / G) >= count) break;  // uniform over the workgroup
      row_block<G, C, MODE>(d, sk, in[k]);
    }
  } else {
#pragma unroll 1
    for (int k = 0; k < REP; ++k) {
      int vb = lblock * REP + k;
      if (vb * (PSL_BLOCK / G) >= count) break;  // uniform over the workgroup
      RowIn<C> in;
      row_entry<G, C>(d, bin, vb, in);
      row_data<G, C>(d, in);
      load_els<C>(d, in.s0, in.len, gl * C, true, in.e);
      row_block<G, C, MODE>(d, sk, in);
    }
  }
}

// ---------------------------------------------------------------------------
// long rows: workgroup passes of 2048 positions (8 contiguous per thread)
// ---------------------------------------------------------------------------

// sums of one pass: (w0 + w1) + (w2 + w3) over the wavefront butterflies
template <int MODE>
__device__ __forceinline__ void pass_stats(const Dev& d, int64_t s0, int len, int base, El (&e)[8], double* wl,
                                           int* il, double& psmin, double& psmax, int& nmin, int& nmax, int& L) {
  double a, b;
  int c;
  lane_stats<8, MODE>(d, s0, len, base + (int)threadIdx.x * 8, e, a, b, c);
  a = group_sum<PSL_WAVE>(a);
  b = group_sum<PSL_WAVE>(b);
  c = group_sum_int<PSL_WAVE>(c);
  int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    wl[w] = a;
    wl[4 + w] = b;
    il[w] = c;
  }
  __syncthreads();
  psmin = (wl[0] + wl[1]) + (wl[2] + wl[3]);
  psmax = (wl[4] + wl[5]) + (wl[6] + wl[7]);
  nmin = nmax = L = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    nmin += cnt_min(il[k]);
    nmax += cnt_max(il[k]);
    L += cnt_act(il[k]);
  }
  __syncthreads();
}

// partial statistics of one chunk (its passes combined in tree order)
template <int MODE>
__global__ void __launch_bounds__(PSL_BLOCK) k_long_stats(Dev d) {
  __shared__ double ps[2 * LONG_MAX_PASSES];
  __shared__ double wl[8];
  __shared__ int il[4];
  LongChunk ch = d.lchunk[blockIdx.x];
  int row = ch.row;
  if (!d.row_on[row]) return;
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  int tmin = 0, tmax = 0, tl = 0;
  int np = ch.npass;
  bool tiny = false;  // an active entry with |a| < coef_tol (forcing rows)
  for (int p = 0; p < np; ++p) {
    El e[8];
    double a, b;
    int x, y, z;
    pass_stats<MODE>(d, s0, len, ch.first + p * PASS_LEN, e, wl, il, a, b, x, y, z);
    if (threadIdx.x == 0) {
      ps[p] = a;
      ps[LONG_MAX_PASSES + p] = b;
    }
    tmin += x;
    tmax += y;
    tl += z;
#pragma unroll
    for (int k = 0; k < 8; ++k) tiny = tiny || (el_active(e[k]) && fabs(e[k].a) < d.cfg.coef_tol);
  }
  int any_tiny = __syncthreads_or(tiny ? 1 : 0);
  if (threadIdx.x == 0) {
    LongPart pt;
    pt.smin = tree_inplace(ps, np);
    pt.smax = tree_inplace(ps + LONG_MAX_PASSES, np);
    pt.nmin = tmin;
    pt.nmax = tmax;
    pt.L = tl;
    pt.tiny = any_tiny ? 1 : 0;
    d.lpart[ch.id] = pt;
  }
}

// row totals from the chunk partials: one wavefront, 8 chunks per lane
__device__ __forceinline__ void long_totals(const Dev& d, const LongRow& lr, RowStat& st, int& L, int& tiny) {
  double a[8], b[8];
  int n0 = 0, n1 = 0, n2 = 0, n3 = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int c = lane_id() * 8 + k;
    a[k] = b[k] = 0.0;
    if (c < lr.nchunk) {
      LongPart pt = d.lpart[lr.chunk0 + c];
      a[k] = pt.smin;
      b[k] = pt.smax;
      n0 += pt.nmin;
      n1 += pt.nmax;
      n2 += pt.L;
      n3 += pt.tiny;
    }
  }
  st.minact = group_sum<PSL_WAVE>(lane_tree<8>(a));
  st.maxact = group_sum<PSL_WAVE>(lane_tree<8>(b));
  st.nmin = group_sum_int<PSL_WAVE>(n0);
  st.nmax = group_sum_int<PSL_WAVE>(n1);
  L = group_sum_int<PSL_WAVE>(n2);
  tiny = group_sum_int<PSL_WAVE>(n3);
}

// decisions and propagation over one chunk of a long row
__device__ __forceinline__ void sweep_long_chunk(const Dev& d, const CandSink& sk, int chunk, double* lds) {
  LongChunk ch = d.lchunk[chunk];
  int row = ch.row;
  if (!d.row_on[row]) {
    if (ch.first == 0 && threadIdx.x == 0) d.row_code[row] = RC_KEEP;
    return;
  }
  LongRow lr = d.lrow[ch.lrow];
  int* li = (int*)(lds + 2);
  if (threadIdx.x < PSL_WAVE) {
    RowStat st;
    int L, tiny;
    long_totals(d, lr, st, L, tiny);
    if (threadIdx.x == 0) {
      lds[0] = st.minact;
      lds[1] = st.maxact;
      li[0] = st.nmin;
      li[1] = st.nmax;
      li[2] = L;
      li[3] = tiny;
    }
  }
  __syncthreads();
  RowStat st;
  st.minact = lds[0];
  st.maxact = lds[1];
  st.nmin = li[0];
  st.nmax = li[1];
  int L = li[2];
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  double lhs = d.lhs[row], rhs = d.rhs[row];
  RowDec dec = decide_row(d.cfg, lhs, rhs, L, st.nmin, st.nmax, st.minact, st.maxact, li[3] != 0);
  if (ch.first == 0 && threadIdx.x == 0) d.rinf[row] = make_int2(st.nmin, st.nmax);
  bool uncap = false, mine = false;
  int aj = 0;
  double aa = 0.0;
  for (int p = 0; p < ch.npass; ++p) {
    int base = ch.first + p * PASS_LEN + (int)threadIdx.x * 8;
    if (dec.prop)
      lane_prop_stream<8>(d, sk, row, true, s0, len, base, lhs, rhs, st, dec.single, dec.force, uncap, mine, aj, aa);
    if (dec.code == RC_REDUNDANT || is_forcing(dec.code)) lane_drop_stream<8>(d, true, s0, len, base, lhs, rhs);
  }
  if (dec.prop && dec.single && !dec.infeasible) {
    // the one active entry decides whether its row becomes bounds
    if (mine) {
      if (!uncap) {
        d.row_code[row] = RC_SINGLETON;
        d.row_out[row] = RowOut{aa, 0.0, aj, 0};
        drop_col(d, aj, aa, lhs, rhs);
      } else {
        d.row_code[row] = RC_KEEP;
      }
    }
  } else if (ch.first == 0 && threadIdx.x == 0) {
    d.row_code[row] = dec.code;
    if (dec.infeasible) flag_infeasible(d, row_lp_of(d, row));
    if (dec.code == RC_EMPTY || dec.code == RC_REDUNDANT || is_forcing(dec.code))
      d.row_out[row] = row_out_of(dec.code, st);
  }
}

__device__ __forceinline__ int long_first_block(const SweepGrid& g) {
  int b = 0;
  for (int k = 0; k < BIN_LONG; ++k) b += g.nb[k];
  return b;
}

// Three launches per sweep, by register need: (0) 4/8/16/64-lane group bins
// with one position per lane, (1) wavefront bins with 4 or 8 positions per
// lane, (2) long-row chunks. Workgroups keep one global numbering across the
// launches (candidate regions and counts are indexed by it).
enum { KIND_SHORT = 0, KIND_WIDE = 1, KIND_LONG = 2, KIND_ALL = 3 };

template <int MODE, int KIND>
__global__ void __launch_bounds__(PSL_BLOCK) k_sweep(Dev d, SweepGrid g, int base) {
  __shared__ double lds[8];
  __shared__ int32_t lcount;
  if (threadIdx.x == 0) lcount = 0;
  __syncthreads();
  int gb = blockIdx.x + base;  // global workgroup number
  int b = gb;
  int bin;
  int64_t start = cand_region_start(g, b, bin);
  int lfb = long_first_block(g);
  if (MODE == MODE_ROUND && (KIND == KIND_LONG || (KIND == KIND_ALL && b >= lfb)))
    start = g.long_base + (int64_t)d.lchunk[b - lfb].cand_off;
  CandSink sk{d.cand + (start < 0 ? 0 : start), &lcount};
  if (KIND == KIND_ALL) {
    if (b < g.nb[BIN_G4]) {
      sweep_rows<4, 1, MODE, 4>(d, sk, BIN_G4, b);
    } else if ((b -= g.nb[BIN_G4]) < g.nb[BIN_G8]) {
      sweep_rows<8, 1, MODE, 4>(d, sk, BIN_G8, b);
    } else if ((b -= g.nb[BIN_G8]) < g.nb[BIN_G16]) {
      sweep_rows<16, 1, MODE, 4>(d, sk, BIN_G16, b);
    } else if ((b -= g.nb[BIN_G16]) < g.nb[BIN_W1]) {
      sweep_rows<64, 1, MODE, 2>(d, sk, BIN_W1, b);
    } else if ((b -= g.nb[BIN_W1]) < g.nb[BIN_W4]) {
      sweep_rows<64, 4, MODE, 1>(d, sk, BIN_W4, b);
    } else if ((b -= g.nb[BIN_W4]) < g.nb[BIN_W8]) {
      sweep_rows<64, 8, MODE, 1>(d, sk, BIN_W8, b);
    } else if (MODE == MODE_ROUND) {
      sweep_long_chunk(d, sk, gb - lfb, lds);
    }
  } else if (KIND == KIND_SHORT) {
    if (b < g.nb[BIN_G4]) {
      sweep_rows<4, 1, MODE, 4>(d, sk, BIN_G4, b);
    } else if ((b -= g.nb[BIN_G4]) < g.nb[BIN_G8]) {
      sweep_rows<8, 1, MODE, 4>(d, sk, BIN_G8, b);
    } else if ((b -= g.nb[BIN_G8]) < g.nb[BIN_G16]) {
      sweep_rows<16, 1, MODE, 4>(d, sk, BIN_G16, b);
    } else {
      b -= g.nb[BIN_G16];
      sweep_rows<64, 1, MODE, 2>(d, sk, BIN_W1, b);
    }
  } else if (KIND == KIND_WIDE) {
    b -= g.nb[BIN_G4] + g.nb[BIN_G8] + g.nb[BIN_G16] + g.nb[BIN_W1];
    if (b < g.nb[BIN_W4]) sweep_rows<64, 4, MODE, 1>(d, sk, BIN_W4, b);
    else sweep_rows<64, 8, MODE, 1>(d, sk, BIN_W8, b - g.nb[BIN_W4]);
  } else if (MODE == MODE_ROUND) {
    sweep_long_chunk(d, sk, b - lfb, lds);
  }
  if (MODE == MODE_ROUND) {
    __syncthreads();
    if (threadIdx.x == 0) d.cand_cnt[gb] = lcount;
  }
}

// compaction: a long row's constant and active length from its partials
__global__ void __launch_bounds__(PSL_BLOCK) k_long_finish_compact(Dev d) {
  int k = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6);
  if (k >= d.nlong) return;
  LongRow lr = d.lrow[k];
  bool on = d.row_on[lr.row] != 0;
  RowStat st;
  int L = 0;
  int tiny = 0;
  if (on) long_totals(d, lr, st, L, tiny);
  else st.minact = 0.0;
  if (lane_id() == 0) {
    d.row_out[lr.row].v0 = st.minact;
    d.row_out[lr.row].j = on ? L : 0;
  }
}

// ---------------------------------------------------------------------------
// source rows of the final bounds
// ---------------------------------------------------------------------------
// one workgroup per sweep workgroup: its candidate region
__global__ void __launch_bounds__(PSL_BLOCK) k_src(Dev d, SweepGrid g) {
  int b = blockIdx.x;
  int n = d.cand_cnt[b];
  if (n == 0) return;
  int bin;
  int64_t start = cand_region_start(g, b, bin);
  if (start < 0) start = g.long_base + (int64_t)d.lchunk[b - long_first_block(g)].cand_off;
  const Cand* list = d.cand + start;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    Cand c = list[i];
    d.touch[c.js >> 1] = 1;
    if (c.t == dunkey(d.bkey[c.js])) atomicMin(&d.src[c.js], c.pos);
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

// decision of an active or removed column from the round's accumulators:
// code bits, and the number of records it gives
// Dual fixing (a lock-based dual reduction): when no alive row keeps column
// j from moving towards the bound its cost prefers (c > 0: down, c < 0: up;
// c = 0: either, with a finite bound, lower first), some optimal solution has
// it there; an infinite such bound means the LP is unbounded if feasible.
// Returns true with the value (possibly infinite) and side (0 lower, 1 upper).
__device__ __forceinline__ bool dual_fix_of(double c, double lo, double up, unsigned long long locks, double& v,
                                            int& side) {
  bool free_down = (locks & 0xFFFFFFFFull) == 0, free_up = (locks >> 32) == 0;
  side = 0;
  v = lo;
  if (c > 0) return free_down;
  side = 1;
  v = up;
  if (c < 0) return free_up;
  if (free_down && !is_inf(lo)) {
    side = 0;
    v = lo;
    return true;
  }
  return free_up && !is_inf(up);
}

__device__ __forceinline__ uint8_t col_decide(const Dev& d, int j, int& k) {
  k = 0;
  double2 b = d.bnd[j];
  if (b.x == b.y) return 0;
  double lo = dunkey(d.bkey[2 * (int64_t)j]);
  double up = dunkey(d.bkey[2 * (int64_t)j + 1]);
  uint8_t code = 0;
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
  } else if (d.cfg.dual_fix) {
    double v;
    int side;
    if (dual_fix_of(d.c[j], lo, up, d.locks[j], v, side)) {
      if (is_inf(v)) {
        code |= CC_UNBOUNDED;
      } else {
        code |= CC_DUALFIX;
        ++k;
      }
    }
  }
  if (code & CC_INFEAS) flag_infeasible(d, col_lp_of(d, j));
  if (code & CC_UNBOUNDED) flag_unbounded(d, col_lp_of(d, j));
  return code;
}

// Decision tiles: the rows in tiles of DEC_TILE, then the columns in tiles of
// DEC_TILE (index order, so the records keep the order rows, then columns).
// A lane loads the codes of DEC_ITEMS consecutive indices as one word (the
// arrays are 256-byte aligned and padded, so a word starting below the end
// stays inside them); the indices with work (touched columns, indices with
// records) are then compacted per wavefront in LDS and dealt out to its lanes,
// so the lanes stay busy whether few or all indices have work, and a tile
// costs four wavefronts instead of one per 64 indices.
#define DEC_ITEMS 4
#define DEC_BLOCK 256
#define DEC_TILE (DEC_BLOCK * DEC_ITEMS)
#define DEC_WAVES (DEC_BLOCK / PSL_WAVE)
#define DEC_WAVE_ITEMS (PSL_WAVE * DEC_ITEMS)
// an index has at most 3 records (a row 1; a column: each bound side and one
// of fixed, empty or dual-fixed), so a lane's count fits in 4 bits
static_assert(3 * DEC_ITEMS < 16, "record counts per lane must fit in 4 bits");
static_assert(DEC_ITEMS == 4, "a lane's codes are one 32-bit word");

// prefix (lanes below) and total of per-lane counts 0..15 across the
// wavefront, from one ballot per bit
__device__ __forceinline__ void wave_small_scan(int v, int& pre, int& tot) {
  unsigned long long below = (1ull << lane_id()) - 1ull;
  unsigned long long b0 = __ballot(v & 1), b1 = __ballot(v & 2), b2 = __ballot(v & 4), b3 = __ballot(v & 8);
  pre = __popcll(b0 & below) + 2 * __popcll(b1 & below) + 4 * __popcll(b2 & below) + 8 * __popcll(b3 & below);
  tot = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2) + 8 * __popcll(b3);
}

// bytes of a lane's word that hold indices below the end (rem of them)
__device__ __forceinline__ uint32_t valid_bytes(int64_t rem) {
  return rem >= 4 ? 0xFFFFFFFFu : (1u << (8 * (int)rem)) - 1u;
}

// the codes' word of a lane: 4 consecutive indices from i0 (a multiple of 4)
__device__ __forceinline__ uint32_t code_word(const uint8_t* a, int64_t i0) {
  return reinterpret_cast<const uint32_t*>(a)[i0 >> 2];
}

// records of a column with decision code `code`
__device__ __forceinline__ int col_recs(uint32_t code) {
  return (code & CC_LB ? 1 : 0) + (code & CC_UB ? 1 : 0) + (code & (CC_FIX | CC_EMPTY) ? 1 : 0);
}

// Column decisions of the touched columns (untouched ones cannot change: an
// active column with unchanged bounds and rows is neither fixed nor empty),
// and the record count of each tile.
__global__ void __launch_bounds__(DEC_BLOCK) k_decide_count(Dev d, int32_t* tile_sum, int64_t row_tiles) {
  __shared__ int list[DEC_TILE];
  __shared__ int wtot[DEC_WAVES];
  int w = threadIdx.x >> 6, lane = lane_id();
  int* wl = list + w * DEC_WAVE_ITEMS;
  int64_t tile = blockIdx.x;
  int c = 0, nt = 0, ntot = 0;
  if (tile < row_tiles) {
    int64_t i0 = tile * DEC_TILE + (int64_t)threadIdx.x * DEC_ITEMS;
    if (i0 < d.m) {
      uint32_t cw = code_word(d.row_code, i0) & valid_bytes(d.m - i0);
#pragma unroll
      for (int b = 0; b < 4; ++b) c += ((cw >> (8 * b)) & 0xFFu) != RC_KEEP;
    }
  } else {
    int64_t j0 = (tile - row_tiles) * DEC_TILE + (int64_t)threadIdx.x * DEC_ITEMS;
    uint32_t tw = 0;
    if (j0 < d.n) {
      uint32_t vm = valid_bytes(d.n - j0);
      uint32_t traw = code_word(d.touch, j0);
      tw = traw & vm;
      uint32_t cw = code_word(d.col_code, j0) & vm;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        bool touched = ((tw >> (8 * b)) & 0xFFu) != 0;
        nt += touched;
        // a code left from an earlier round of an untouched column
        if (!touched && ((cw >> (8 * b)) & 0xFFu)) d.col_code[j0 + b] = 0;
      }
      if (tw) reinterpret_cast<uint32_t*>(d.touch)[j0 >> 2] = traw & ~vm;
    }
    // the touched columns of the wavefront, in LDS, dealt out to its lanes
    int pre;
    wave_small_scan(nt, pre, ntot);
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if ((tw >> (8 * b)) & 0xFFu) wl[pre++] = (int)(j0 + b);
  }
  __syncthreads();
  for (int e = lane; e < ntot; e += PSL_WAVE) {
    int j = wl[e];
    int kk;
    d.col_code[j] = col_decide(d, j, kk);
    c += kk;
  }
  // the tile's record count: wavefront totals by ballots, summed by thread 0
  int pre_w, tot_w;
  wave_small_scan(c, pre_w, tot_w);
  if (lane == 0) wtot[w] = tot_w;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
#pragma unroll
    for (int k = 0; k < DEC_WAVES; ++k) tot += wtot[k];
    tile_sum[tile] = tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.flags->rows_removed = 0;
    d.flags->fin_cols = 0;
  }
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

__device__ __forceinline__ void emit_row(const Dev& d, int i, int round, Record* r) {
  uint8_t code = d.row_code[i];
  RowOut o = d.row_out[i];
  if (code == RC_EMPTY) *r = mkrec(REC_EMPTY_ROW, 0, round, i, -1, -1, o.v0, d.lhs[i], d.rhs[i], 0.0);
  else if (code == RC_REDUNDANT) *r = mkrec(REC_REDUNDANT_ROW, 0, round, i, -1, -1, o.v0, o.v1, d.lhs[i], d.rhs[i]);
  else if (is_forcing(code))
    *r = mkrec(REC_FORCING_ROW, code == RC_FORCE_MAX ? 1 : 0, round, i, -1, -1, o.v0, d.lhs[i], d.rhs[i], 0.0);
  else *r = mkrec(REC_SINGLETON_ROW, 0, round, i, o.j, -1, o.v0, d.lhs[i], d.rhs[i], 0.0);
  d.row_on[i] = 0;
  d.row_code[i] = RC_KEEP;
}

// returns 1 when a bound of the column became finite
__device__ __forceinline__ int emit_col(const Dev& d, int j, int round, Record* r) {
  uint8_t code = d.col_code[j];
  double2 b = d.bnd[j];
  double lo = dunkey(d.bkey[2 * (int64_t)j]);
  double up = dunkey(d.bkey[2 * (int64_t)j + 1]);
  // the source of a changed bound is the CSR position of the lowest row's
  // candidate equal to it (positions of one column ascend with the row); a
  // changed bound always has one
  if (code & CC_LB) {
    int q = d.src[2 * (int64_t)j];
    bool ok = q >= 0 && q < d.nnz;
    int k = ok ? d.rowid1[q + 1] : -1;
    *r++ = mkrec(REC_BOUND_CHANGE, 0, round, -1, j, k, b.x, lo, ok ? d.va[q] : __builtin_nan(""), 0.0);
    int ls = d.lsrc[j];
    d.lsrc[j] = ls == -1 || ls == k ? k : -2;  // a bound from one row only keeps it implied by that row
  }
  if (code & CC_UB) {
    int q = d.src[2 * (int64_t)j + 1];
    bool ok = q >= 0 && q < d.nnz;
    int k = ok ? d.rowid1[q + 1] : -1;
    *r++ = mkrec(REC_BOUND_CHANGE, 1, round, -1, j, k, b.y, up, ok ? d.va[q] : __builtin_nan(""), 0.0);
    int us = d.usrc[j];
    d.usrc[j] = us == -1 || us == k ? k : -2;
  }
  double nlo = lo, nup = up;
  if ((code & CC_DUALFIX) == CC_DUALFIX) {
    // the locks have not changed since the decision
    double v;
    int side;
    dual_fix_of(d.c[j], lo, up, d.locks[j], v, side);
    *r++ = mkrec(REC_DUAL_FIX, (uint8_t)side, round, -1, j, -1, v, d.c[j], 0.0, 0.0);
    nlo = nup = v;
  } else if (code & CC_FIX) {
    *r++ = mkrec(REC_FIX_COL, 0, round, -1, j, -1, lo, d.c[j], 0.0, 0.0);
    nlo = nup = lo;
  } else if (code & CC_EMPTY) {
    double v = empty_value(d.c[j], lo, up);
    *r++ = mkrec(REC_EMPTY_COL, 0, round, -1, j, -1, v, d.c[j], 0.0, 0.0);
    nlo = nup = v;
  }
  // bounds that became finite lower the infinite-contribution counts of
  // the column's rows (applied by the marking pass)
  uint8_t fin = (is_inf(b.x) && !is_inf(nlo) ? CC_LBFIN : 0) | (is_inf(b.y) && !is_inf(nup) ? CC_UBFIN : 0);
  if (fin) d.col_code[j] = code | fin;
  d.bnd[j] = make_double2(nlo, nup);
  d.bkey[2 * (int64_t)j] = dkey(nlo);
  d.bkey[2 * (int64_t)j + 1] = dkey(nup);
  d.src[2 * (int64_t)j] = 0x7FFFFFFF;
  d.src[2 * (int64_t)j + 1] = 0x7FFFFFFF;
  return fin ? 1 : 0;
}

// Records of the round in index order: each tile's offset comes from the
// scanned tile sums, the position of an index's records inside the tile from
// the counts of the indices before it (ballots inside the wavefront, the
// wavefronts' totals through LDS). The indices with records are compacted per
// wavefront and dealt out to its lanes, each writing its index's records at
// that position. Also sets the rows removed and (batches) marks the LPs that
// changed.
__global__ void __launch_bounds__(DEC_BLOCK) k_decide_emit(Dev d, const int32_t* tile_sum, const int32_t* tile_off,
                                                            int64_t row_tiles, int64_t base, int round) {
  int64_t tile = blockIdx.x;
  // a row tile's records are its removed rows, so the rows removed are the
  // records before the first column tile (the scanned tile sums)
  if (tile == 0 && threadIdx.x == 0)
    d.flags->rows_removed = row_tiles < (int64_t)gridDim.x ? tile_off[row_tiles] : d.flags->round_total;
  int tsum = tile_sum[tile];
  if (tsum == 0) return;  // a tile without records
  __shared__ int list[DEC_TILE], lpos[DEC_TILE];
  __shared__ int wtot[DEC_WAVES], wfin[DEC_WAVES];
  int w = threadIdx.x >> 6, lane = lane_id();
  bool rows = tile < row_tiles;
  int64_t t0 = (rows ? tile : tile - row_tiles) * DEC_TILE + (int64_t)threadIdx.x * DEC_ITEMS;
  int64_t lim = rows ? d.m : d.n;
  uint32_t cnt4 = 0;  // the records of the lane's 4 indices, a byte each
  if (t0 < lim) {
    uint32_t vm = valid_bytes(lim - t0);
    uint32_t cw = code_word(rows ? d.row_code : d.col_code, t0) & vm;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t code = (cw >> (8 * b)) & 0xFFu;
      cnt4 |= (uint32_t)(rows ? code != RC_KEEP : col_recs(code)) << (8 * b);
    }
  }
  int c = 0, ni = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int k = (cnt4 >> (8 * b)) & 0xFF;
    c += k;
    ni += k != 0;
  }
  int pre, tot_w, ipre, itot;
  wave_small_scan(c, pre, tot_w);
  wave_small_scan(ni, ipre, itot);
  if (lane == 0) wtot[w] = tot_w;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < DEC_WAVES; ++k) pre += k < w ? wtot[k] : 0;
  int* wl = list + w * DEC_WAVE_ITEMS;
  int* wp = lpos + w * DEC_WAVE_ITEMS;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int k = (cnt4 >> (8 * b)) & 0xFF;
    if (k) {
      wl[ipre] = (int)(t0 + b);
      wp[ipre] = pre;
      ++ipre;
      pre += k;
    }
  }
  __syncthreads();
  Record* r0 = d.rec + base + tile_off[tile];
  int fin = 0;
  for (int e = lane; e < itot; e += PSL_WAVE) {
    int x = wl[e];
    Record* r = r0 + wp[e];
    int lp;
    if (rows) {
      lp = row_lp_of(d, x);
      emit_row(d, x, round_of(d, lp, round), r);
    } else {
      lp = col_lp_of(d, x);
      fin += emit_col(d, x, round_of(d, lp, round), r);
    }
    if (d.K > 1) d.lpo[lp].total = 1;  // the LP changed this round
  }
  if (rows) return;
  // columns whose bound became finite: one atomic per workgroup
  int fpre, ftot_w;
  wave_small_scan(fin, fpre, ftot_w);
  if (lane == 0) wfin[w] = ftot_w;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ftot = 0;
#pragma unroll
    for (int k = 0; k < DEC_WAVES; ++k) ftot += wfin[k];
    if (ftot) atomicAdd(&d.flags->fin_cols, ftot);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_long_stats(const Dev& d, int mode, hipStream_t s) {
  if (d.nchunks == 0) return;
  if (mode == MODE_ROUND) hipLaunchKernelGGL(k_long_stats<MODE_ROUND>, dim3(d.nchunks), dim3(PSL_BLOCK), 0, s, d);
  else hipLaunchKernelGGL(k_long_stats<MODE_COMPACT>, dim3(d.nchunks), dim3(PSL_BLOCK), 0, s, d);
}

void launch_sweep(const Dev& d, const SweepGrid& g, int mode, hipStream_t s) {
  int n_short = g.nb[BIN_G4] + g.nb[BIN_G8] + g.nb[BIN_G16] + g.nb[BIN_W1];
  int n_wide = g.nb[BIN_W4] + g.nb[BIN_W8];
  int n_long = g.nb[BIN_LONG];
  if (mode == MODE_ROUND) {
    int total = n_short + n_wide + n_long;
    if (total) hipLaunchKernelGGL((k_sweep<MODE_ROUND, KIND_ALL>), dim3(total), dim3(PSL_BLOCK), 0, s, d, g, 0);
  } else if (mode == 2) {
    if (n_short) hipLaunchKernelGGL((k_sweep<MODE_ROUND, KIND_SHORT>), dim3(n_short), dim3(PSL_BLOCK), 0, s, d, g, 0);
    if (n_wide)
      hipLaunchKernelGGL((k_sweep<MODE_ROUND, KIND_WIDE>), dim3(n_wide), dim3(PSL_BLOCK), 0, s, d, g, n_short);
    if (n_long)
      hipLaunchKernelGGL((k_sweep<MODE_ROUND, KIND_LONG>), dim3(n_long), dim3(PSL_BLOCK), 0, s, d, g,
                         n_short + n_wide);
  } else {
    if (n_short)
      hipLaunchKernelGGL((k_sweep<MODE_COMPACT, KIND_SHORT>), dim3(n_short), dim3(PSL_BLOCK), 0, s, d, g, 0);
    if (n_wide)
      hipLaunchKernelGGL((k_sweep<MODE_COMPACT, KIND_WIDE>), dim3(n_wide), dim3(PSL_BLOCK), 0, s, d, g, n_short);
    if (d.nlong > 0)
      hipLaunchKernelGGL(k_long_finish_compact, dim3((d.nlong + 3) / 4), dim3(PSL_BLOCK), 0, s, d);
  }
}

// every long row's removed-column constant and active length (row_out), from
// the compaction-mode chunk partials
void launch_long_consts(const Dev& d, hipStream_t s) {
  if (d.nlong == 0) return;
  launch_long_stats(d, MODE_COMPACT, s);
  hipLaunchKernelGGL(k_long_finish_compact, dim3((d.nlong + 3) / 4), dim3(PSL_BLOCK), 0, s, d);
}

void launch_src(const Dev& d, const SweepGrid& g, hipStream_t s) {
  int total = 0;
  for (int b = 0; b < NBINS; ++b) total += g.nb[b];
  if (total > 0) hipLaunchKernelGGL(k_src, dim3(total), dim3(PSL_BLOCK), 0, s, d, g);
}

// the round's decisions and records: counts per tile, scan, emission; the
// record total goes to d.flags->round_total
void launch_decide(const Dev& d, int64_t base, int round, int32_t* tile_sum, int32_t* tile_off, int32_t* ws,
                   hipStream_t s) {
  int64_t row_tiles = ((int64_t)d.m + DEC_TILE - 1) / DEC_TILE;
  int64_t tiles = row_tiles + ((int64_t)d.n + DEC_TILE - 1) / DEC_TILE;
  if (tiles == 0) {
    fill_i32(&d.flags->round_total, 0, 1, s);
    fill_i32(&d.flags->rows_removed, 0, 1, s);
    return;
  }
  hipLaunchKernelGGL(k_decide_count, dim3((unsigned)tiles), dim3(DEC_BLOCK), 0, s, d, tile_sum, row_tiles);
  scan_excl(tile_sum, tile_off, tiles, &d.flags->round_total, ws, s);
  hipLaunchKernelGGL(k_decide_emit, dim3((unsigned)tiles), dim3(DEC_BLOCK), 0, s, d, (const int32_t*)tile_sum,
                     (const int32_t*)tile_off, row_tiles, base, round);
}

int long_max_passes() { return LONG_MAX_PASSES; }

}  // namespace psl
