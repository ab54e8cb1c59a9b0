// parallel.hip -- parallel rows (section 3.2, "Parallel rows") of the
// current problem: columns that are fixed or removed are ignored, as when A
// is streamed (section 3.2, "Internal data structures").
//
// Two rows are parallel when a_i = lambda a_k over their active entries.
// Every active row with at least two active columns is hashed independently
// (two levels: the active sparsity pattern, then the active coefficients
// normalised by the row's first active coefficient and quantised), the keys
// go into an open-addressing table, and each row of a key group is checked
// against the group's leader: the lowest equality row of the group, else its
// lowest row. The hash pass also leaves every live row's removed-column
// constant k_i (canonical pairwise sum over its positions; long rows from
// their chunk partials) and active length in row_out. Sides are compared in the
// effective frame [lhs - k, rhs - k]: verified rows are removed and the
// leader's effective sides become the intersection of the mapped sides; the
// row giving each final side is the lowest such row. A side the leader keeps
// keeps its stored value, one taken from another row is stored as
// effective + k_leader.
#include "bits.h"
#include "psl_kern.h"
#include "sweep.h"

namespace psl {

// col0: first column of the row's LP (the pattern is hashed in the LP's own
// column numbering, so a row's key does not depend on its place in a batch).
// Only active entries (column bounds not equal) enter the key; whether a
// column is active comes from the pass's bit array (one bit per column, in
// L2), and only a fixed column's entry reads its bounds (for the constant).
__device__ __forceinline__ void hash_el(int j, double a, bool act, double a0, int col0, unsigned long long& h1,
                                        unsigned long long& h2) {
  unsigned long long cj = splitmix((unsigned long long)(uint32_t)(j - col0));
  h1 = act ? cj : 0ULL;
  h2 = act ? splitmix(cj ^ quantize(a / a0)) : 0ULL;
}

// Hash terms of the positions q = q0 + u * STRIDE + lane (u < U, valid when
// q < end) of a row starting at s0 (which is a valid position: the row has
// entries), added to s1 / s2, active ones counted in L. All loads are issued
// before any is used.
template <int U, int STRIDE>
__device__ __forceinline__ void hash_batch(const Dev& d, const uint64_t* abits, int64_t s0, int q0, int lane, int end,
                                           double a0, int col0, unsigned long long& s1, unsigned long long& s2,
                                           int& L) {
  int j[U];
  double a[U];
  bool v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    int q = q0 + u * STRIDE + lane;
    v[u] = q < end;
    int64_t p = v[u] ? s0 + q : s0;
    j[u] = d.ci[p];
    a[u] = d.va[p];
  }
  bool act[U];
#pragma unroll
  for (int u = 0; u < U; ++u) act[u] = v[u] && bit_of(abits, j[u]);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    unsigned long long h1, h2;
    hash_el(j[u], a[u], act[u], a0, col0, h1, h2);
    s1 += h1;
    s2 += h2;
    L += act[u] ? 1 : 0;
  }
}

// First active position of a row (one wavefront, all lanes return it), or
// -1 when no column of the row is active.
__device__ __forceinline__ int first_active_pos(const Dev& d, const uint64_t* abits, int64_t s0, int len) {
  int lane = lane_id();
  for (int q0 = 0; q0 < len; q0 += PSL_WAVE) {
    int q = q0 + lane;
    bool act = q < len && bit_of(abits, d.ci[s0 + q]);
    unsigned long long mask = __ballot(act);
    if (mask) return q0 + __ffsll((long long)mask) - 1;
  }
  return -1;
}

__device__ __forceinline__ unsigned long long row_key(int len, unsigned long long s1, unsigned long long s2) {
  return (splitmix((unsigned long long)len + s1) ^ s2) | 1ULL;
}

__device__ __forceinline__ int lp_col0(const Dev& d, int row) { return d.K > 1 ? d.lp_col0[d.row_lp[row]] : 0; }

// a stored side of live row i in the frame of its active columns: moved by
// the removed columns' constant (row_out[i].v0, from the hash pass);
// infinite sides stay
__device__ __forceinline__ double eff_side(const Dev& d, int i, double side) {
  return is_inf(side) ? side : pos0(side - d.row_out[i].v0);
}

// every LP has its own table (a power-of-two slice of the slot array), so key
// groups never mix rows of different LPs
__device__ __forceinline__ void par_insert(const Dev& d, const ParScratch& P, int row, unsigned long long key) {
  int64_t base = 0, cap = P.cap;
  if (d.K > 1) {
    LpTab t = P.lpt[d.row_lp[row]];
    base = t.base;
    cap = t.cap;
  }
  HashSlot* tab = P.table + base;
  unsigned long long mask = (unsigned long long)cap - 1;
  unsigned long long h = splitmix(key) & mask;
  for (int64_t probe = 0; probe < cap; ++probe) {
    unsigned long long old = atomicCAS(&tab[h].key, 0ULL, key);
    if (old == 0ULL || old == key) break;
    h = (h + 1) & mask;
  }
  bool eq = d.lhs[row] == d.rhs[row];
  atomicMin(&tab[h].leader, (eq ? 0u : 0x80000000u) | (unsigned)row);
  P.slot[row] = (int)(base + (int64_t)h);
}

// R rows' inserts of one lane: the first compare-and-swap of each is issued
// before any result is used (their latencies overlap); a row whose home slot
// holds another key probes on as par_insert does
template <int R>
__device__ __forceinline__ void par_insert_n(const Dev& d, const ParScratch& P, const int (&row)[R],
                                             const unsigned long long (&key)[R], const bool (&ins)[R]) {
  HashSlot* tab[R];
  unsigned long long mask[R], h[R], old[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    int64_t base = 0, cap = P.cap;
    if (ins[k] && d.K > 1) {
      LpTab t = P.lpt[d.row_lp[row[k]]];
      base = t.base;
      cap = t.cap;
    }
    tab[k] = P.table + base;
    mask[k] = (unsigned long long)cap - 1;
    h[k] = splitmix(key[k]) & mask[k];
  }
#pragma unroll
  for (int k = 0; k < R; ++k) old[k] = ins[k] ? atomicCAS(&tab[k][h[k]].key, 0ULL, key[k]) : 0ULL;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (!ins[k]) continue;
    unsigned long long o = old[k];
    for (unsigned long long probe = 1; o != 0ULL && o != key[k] && probe <= mask[k]; ++probe) {
      h[k] = (h[k] + 1) & mask[k];
      o = atomicCAS(&tab[k][h[k]].key, 0ULL, key[k]);
    }
    bool eq = d.lhs[row[k]] == d.rhs[row[k]];
    atomicMin(&tab[k][h[k]].leader, (eq ? 0u : 0x80000000u) | (unsigned)row[k]);
    P.slot[row[k]] = (int)((tab[k] - P.table) + (int64_t)h[k]);
  }
}

__global__ void k_par_reset(Dev d, ParScratch P) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P.cap; t += stride) {
    HashSlot z;
    z.key = 0;
    z.leader = 0xFFFFFFFFu;
    z.pad = 0;
    P.table[t] = z;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += stride) {
    P.slot[i] = -1;
    P.lead[i] = -1;
    P.is_leader[i] = 0;
    P.side_src[2 * i] = 0x7FFFFFFF;
    P.side_src[2 * i + 1] = 0x7FFFFFFF;
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 4 * (int64_t)d.nlong; k += stride)
    P.hacc[k] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.flags->vlist_count = 0;
    d.flags->merged = 0;
    d.flags->lead_count = 0;
  }
}

// G-lane groups, rows of at most G entries, one position per lane, for REP
// row blocks of the workgroup: the loads of all REP blocks are issued level by
// level (bin entries, then rows and positions, then the active bits and the
// fixed columns' values) before any block is hashed, so a lane has REP rows'
// loads in flight together. A lane without a row reads the bin's first entry
// (which exists) and position 0 or the row's first position, so no load of a
// level is conditional; the first active coefficient comes from the lowest
// active lane of the group.
template <int G, int REP>
__device__ __forceinline__ void hash_groups(const Dev& d, const ParScratch& P, int bin, int lblock0) {
  const int per_block = PSL_BLOCK / G;
  int count = d.bin_off[bin + 1] - d.bin_off[bin];
  int gl = threadIdx.x & (G - 1);
  int row[REP], len[REP];
  int64_t p[REP];
  bool vr[REP];
#pragma unroll
  for (int k = 0; k < REP; ++k) {
    int gid = (lblock0 + k) * per_block + (int)(threadIdx.x / G);
    vr[k] = gid < count;
    BinEnt be = d.bins[d.bin_off[bin] + (vr[k] ? gid : 0)];
    row[k] = be.row;
    len[k] = vr[k] ? be.len : 0;
    int64_t p0 = len[k] > 0 ? be.start : 0;
    p[k] = gl < len[k] ? be.start + gl : p0;
  }
  bool on[REP];
  int j[REP];
  double a[REP];
#pragma unroll
  for (int k = 0; k < REP; ++k) {
    on[k] = vr[k] && d.row_on[row[k]] != 0;
    j[k] = d.ci[p[k]];
    a[k] = d.va[p[k]];
  }
  bool in_row[REP], act0[REP];
  double xf[REP];  // a fixed column's value
#pragma unroll
  for (int k = 0; k < REP; ++k) {
    in_row[k] = on[k] && gl < len[k];
    act0[k] = in_row[k] && bit_of(P.abits, j[k]);
    xf[k] = 0.0;
    if (in_row[k] && !act0[k]) xf[k] = d.bnd[j[k]].x;
  }
  unsigned long long key[REP];
  bool ins[REP];
#pragma unroll
  for (int k = 0; k < REP; ++k) {
    ins[k] = false;
    key[k] = 0;
    if ((lblock0 + k) * per_block >= count) continue;  // uniform over the workgroup
    unsigned long long gmask = __ballot(act0[k]) & group_mask<G>();
    int first = gmask ? __ffsll((long long)gmask) - 1 : lane_id();
    double a0 = __shfl(a[k], first, PSL_WAVE);
    if (!gmask) a0 = 1.0;
    int col0 = lp_col0(d, row[k]);
    unsigned long long h1, h2;
    hash_el(j[k], a[k], act0[k], a0, col0, h1, h2);
    h1 = group_sum_u64<G>(h1);
    h2 = group_sum_u64<G>(h2);
    int L = __popcll(gmask);
    // the removed columns' constant: a butterfly over the group's lanes is the
    // canonical pairwise tree of the row's positions
    double kc = group_sum<G>(in_row[k] && !act0[k] ? pos0(a[k] * xf[k]) : 0.0);
    if (vr[k] && on[k] && gl == 0) {
      d.row_out[row[k]].v0 = kc;
      d.row_out[row[k]].j = L;
      ins[k] = L >= 2;
      key[k] = row_key(L, h1, h2);
    }
  }
  par_insert_n<REP>(d, P, row, key, ins);
}

// pairwise tree over C values held in registers (C a power of two)
template <int C>
__device__ __forceinline__ double reg_tree(double (&x)[C]) {
#pragma unroll
  for (int w = 1; w < C; w <<= 1)
#pragma unroll
    for (int i = 0; i < C; i += 2 * w) x[i] = x[i] + x[i + w];
  return x[0];
}

// One wavefront per row of at most 64 * C entries, C contiguous positions
// per lane (the sweep's layout, so that the lane trees and a butterfly over
// the wavefront give the canonical pairwise tree of the removed columns'
// constant). The first active coefficient is that of the lowest lane with
// an active entry, at its first active position.
template <int C>
__device__ __forceinline__ void hash_wave_row(const Dev& d, const ParScratch& P, int row) {
  int lane = lane_id();
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  if (!d.row_on[row]) return;
  int j[C];
  double a[C];
  bool v[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    int q = lane * C + k;
    v[k] = q < len;
    int64_t p = v[k] ? s0 + q : (len > 0 ? s0 : 0);
    j[k] = d.ci[p];
    a[k] = d.va[p];
  }
  bool act[C];
  double x[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    act[k] = v[k] && bit_of(P.abits, j[k]);
    x[k] = 0.0;
    if (v[k] && !act[k]) x[k] = d.bnd[j[k]].x;  // a fixed column's value
  }
  int lf = C;
  double af = 1.0;
#pragma unroll
  for (int k = C - 1; k >= 0; --k) {
    if (act[k]) {
      lf = k;
      af = a[k];
    }
  }
  unsigned long long mask = __ballot(lf < C);
  double a0 = mask ? __shfl(af, __ffsll((long long)mask) - 1, PSL_WAVE) : 1.0;
  int col0 = lp_col0(d, row);
  unsigned long long s1 = 0, s2 = 0;
  int L = 0;
  double t[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    unsigned long long h1, h2;
    hash_el(j[k], a[k], act[k], a0, col0, h1, h2);
    s1 += h1;
    s2 += h2;
    L += act[k] ? 1 : 0;
    t[k] = v[k] && !act[k] ? pos0(a[k] * x[k]) : 0.0;
  }
  double kc = group_sum<PSL_WAVE>(reg_tree<C>(t));
  s1 = group_sum_u64<PSL_WAVE>(s1);
  s2 = group_sum_u64<PSL_WAVE>(s2);
  L = (int)group_sum_u64<PSL_WAVE>((unsigned long long)L);
  if (lane == 0) {
    d.row_out[row].v0 = kc;
    d.row_out[row].j = L;
    if (L >= 2) par_insert(d, P, row, row_key(L, s1, s2));
  }
}

// long rows: the first active coefficient of each (one wavefront per row),
// kept in the fourth accumulator word (0 when none is active)
__global__ void __launch_bounds__(PSL_BLOCK) k_par_long_first(Dev d, ParScratch P) {
  int k = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6);
  if (k >= d.nlong) return;
  int row = d.lrow[k].row;
  if (!d.row_on[row]) return;
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  int f = first_active_pos(d, P.abits, s0, len);
  if (lane_id() == 0) P.hacc[4 * (int64_t)k + 3] = f < 0 ? 0ull : (unsigned long long)__double_as_longlong(d.va[s0 + f]);
}

// long rows: one workgroup per chunk, accumulated with 64-bit atomic adds
// (the key is a sum modulo 2^64, so the order does not matter)
__device__ __forceinline__ void hash_long_chunk(const Dev& d, const ParScratch& P, int chunk) {
  LongChunk ch = d.lchunk[chunk];
  int row = ch.row;
  if (!d.row_on[row]) return;
  unsigned long long a0b = P.hacc[4 * (int64_t)ch.lrow + 3];
  if (a0b == 0ull) return;  // no active column
  double a0 = __longlong_as_double((long long)a0b);
  int64_t s0 = d.rp[row];
  int len = d.rp[row + 1] - (int)s0;
  int col0 = lp_col0(d, row);
  unsigned long long s1 = 0, s2 = 0;
  int L = 0;
  int end = min(len, ch.first + ch.npass * PASS_LEN);
  for (int q0 = ch.first; q0 < end; q0 += 4 * PSL_BLOCK)
    hash_batch<4, PSL_BLOCK>(d, P.abits, s0, q0, (int)threadIdx.x, end, a0, col0, s1, s2, L);
  s1 = group_sum_u64<PSL_WAVE>(s1);
  s2 = group_sum_u64<PSL_WAVE>(s2);
  unsigned long long l64 = group_sum_u64<PSL_WAVE>((unsigned long long)L);
  if (lane_id() == 0) {
    atomicAdd(&P.hacc[4 * (int64_t)ch.lrow], s1);
    atomicAdd(&P.hacc[4 * (int64_t)ch.lrow + 1], s2);
    atomicAdd(&P.hacc[4 * (int64_t)ch.lrow + 2], l64);
  }
}

// the wavefront rows of a row block (four per workgroup)
__device__ __forceinline__ void hash_wave_block(const Dev& d, const ParScratch& P, int bin, int vb) {
  int wid = vb * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6);
  if (wid >= d.bin_off[bin + 1] - d.bin_off[bin]) return;
  int row = d.bins[d.bin_off[bin] + wid].row;
  if (bin == BIN_W1) hash_wave_row<1>(d, P, row);
  else if (bin == BIN_W4) hash_wave_row<4>(d, P, row);
  else hash_wave_row<8>(d, P, row);
}

// one workgroup per workgroup of the sweep's grid (the same row blocks)
__global__ void __launch_bounds__(PSL_BLOCK) k_par_hash(Dev d, ParScratch P, SweepGrid g) {
  int b = blockIdx.x;
  for (int bin = 0; bin < BIN_LONG; ++bin) {
    if (b >= g.nb[bin]) {
      b -= g.nb[bin];
      continue;
    }
    int rep = bin_rep(bin);
    int count = d.bin_off[bin + 1] - d.bin_off[bin];
    if (bin == BIN_G4) hash_groups<4, 4>(d, P, bin, b * rep);
    else if (bin == BIN_G8) hash_groups<8, 4>(d, P, bin, b * rep);
    else if (bin == BIN_G16) hash_groups<16, 4>(d, P, bin, b * rep);
    else
      for (int k = 0; k < rep; ++k) {
        int vb = b * rep + k;
        if (vb * bin_rows(bin) >= count) break;
        hash_wave_block(d, P, bin, vb);
      }
    return;
  }
  if (b < g.nb[BIN_LONG]) hash_long_chunk(d, P, b);
}

__global__ void k_par_long_insert(Dev d, ParScratch P) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.nlong) return;
  int row = d.lrow[k].row;
  if (!d.row_on[row]) return;
  int64_t L = (int64_t)P.hacc[4 * (int64_t)k + 2];
  if (L >= 2) par_insert(d, P, row, row_key((int)L, P.hacc[4 * (int64_t)k], P.hacc[4 * (int64_t)k + 1]));
}

// rows of a key group other than its leader go to the verify list (a row
// whose slot names another row as leader is in a group of two or more)
// the rows to verify (not their group's leader) appended to P.vlist in any
// order: one counter update per 1024 rows (every row of the 1% that are
// non-leaders would otherwise leave most wavefronts updating one address)
#define VLIST_BLOCK 1024
__global__ void __launch_bounds__(VLIST_BLOCK) k_par_vlist(Dev d, ParScratch P) {
  __shared__ int wcount[VLIST_BLOCK / PSL_WAVE];
  __shared__ int gbase;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool pred = false;
  if (i < d.m) {
    int s = P.slot[i];
    if (s >= 0) {
      pred = (int)(P.table[s].leader & 0x7FFFFFFFu) != (int)i;
      // a possible leader's merged sides start from its own effective ones
      // (its constant is known once the hash pass is done)
      P.side_key[2 * i] = dkey(eff_side(d, (int)i, d.lhs[i]));
      P.side_key[2 * i + 1] = dkey(eff_side(d, (int)i, d.rhs[i]));
    }
  }
  unsigned long long mask = __ballot(pred);
  int w = threadIdx.x >> 6;
  if (lane_id() == 0) wcount[w] = (int)__popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < VLIST_BLOCK / PSL_WAVE; ++k) {
      int c = wcount[k];
      wcount[k] = t;
      t += c;
    }
    gbase = t ? atomicAdd(&d.flags->vlist_count, t) : 0;
  }
  __syncthreads();
  if (pred) P.vlist[gbase + wcount[w] + __popcll(mask & lanemask_lt())] = (int)i;
}

// effective sides of row r mapped through lambda onto its leader's frame
__device__ __forceinline__ void mapped_sides(const Dev& d, int r, double lam, double& ml, double& mu) {
  double lr = eff_side(d, r, d.lhs[r]), rr = eff_side(d, r, d.rhs[r]);
  if (lam > 0) {
    ml = lr / lam;
    mu = rr / lam;
  } else {
    ml = rr / lam;
    mu = lr / lam;
  }
  ml = pos0(ml);
  mu = pos0(mu);
}

// position of column j among positions [s, s + len) of a row (ascending
// columns), or -1
__device__ __forceinline__ int64_t find_col(const Dev& d, int64_t s, int len, int j) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (d.ci[s + mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && d.ci[s + lo] == j ? s + lo : -1;
}

// One wavefront per listed row r: parallel to its leader L when both have
// the same number of active entries and every active entry of r is in L
// (found by binary search in L's ascending columns) with the same value
// after dividing each row by its first active coefficient, within par_tol.
__global__ void __launch_bounds__(PSL_BLOCK) k_par_verify(Dev d, ParScratch P) {
  int nv = d.flags->vlist_count;
  int lane = lane_id();
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int k = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); k < nv; k += wstride) {
    int r = P.vlist[k];
    int L = (int)(P.table[P.slot[r]].leader & 0x7FFFFFFFu);
    int64_t sr = d.rp[r], sl = d.rp[L];
    int len = d.rp[r + 1] - (int)sr, lenL = d.rp[L + 1] - (int)sl;
    bool ok = d.row_out[r].j == d.row_out[L].j;
    int fr = -1, fl = -1;
    if (ok) {
      fr = first_active_pos(d, P.abits, sr, len);
      fl = first_active_pos(d, P.abits, sl, lenL);
      ok = fr >= 0 && fl >= 0;
    }
    double r0 = ok ? d.va[sr + fr] : 1.0, l0 = ok ? d.va[sl + fl] : 1.0;
    for (int q0 = fr; ok && q0 < len; q0 += PSL_WAVE) {
      int q = q0 + lane;
      bool bad = false;
      if (q < len) {
        int j = d.ci[sr + q];
        if (bit_of(P.abits, j)) {
          int64_t pl = find_col(d, sl, lenL, j);
          if (pl < 0) {
            bad = true;
          } else {
            double x = d.va[sr + q] / r0, y = d.va[pl] / l0;
            double scale = fabs(x) > fabs(y) ? fabs(x) : fabs(y);
            bad = !(fabs(x - y) <= d.cfg.par_tol * scale);
          }
        }
      }
      ok = __ballot(bad) == 0;
    }
    if (ok && lane == 0) {
      double lam = r0 / l0, ml, mu;
      mapped_sides(d, r, lam, ml, mu);
      P.lam[r] = lam;
      P.lead[r] = L;
      P.is_leader[L] = 1;
      atomicMax(&P.side_key[2 * (int64_t)L], dkey(ml));
      atomicMin(&P.side_key[2 * (int64_t)L + 1], dkey(mu));
    }
  }
}

// lowest row giving each final side of a leader (the leader counts itself)
__global__ void k_par_src(Dev d, ParScratch P) {
  int nv = d.flags->vlist_count;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nv; k += gridDim.x * blockDim.x) {
    int r = P.vlist[k];
    int L = P.lead[r];
    if (L < 0) continue;
    double ml, mu;
    mapped_sides(d, r, P.lam[r], ml, mu);
    double lo = dunkey(P.side_key[2 * (int64_t)L]);
    double up = dunkey(P.side_key[2 * (int64_t)L + 1]);
    if (ml == lo) atomicMin(&P.side_src[2 * (int64_t)L], r);
    if (mu == up) atomicMin(&P.side_src[2 * (int64_t)L + 1], r);
    if (eff_side(d, L, d.lhs[L]) == lo) atomicMin(&P.side_src[2 * (int64_t)L], L);
    if (eff_side(d, L, d.rhs[L]) == up) atomicMin(&P.side_src[2 * (int64_t)L + 1], L);
  }
}

// The leader's new stored sides (nl, nu) from the merged effective ones;
// returns whether they differ from its current sides.
__device__ __forceinline__ bool leader_sides(const Dev& d, const ParScratch& P, int i, double& nl, double& nu,
                                             bool& infeasible) {
  double lo = dunkey(P.side_key[2 * (int64_t)i]);
  double up = dunkey(P.side_key[2 * (int64_t)i + 1]);
  infeasible = false;
  bool snapped = false;
  if (!is_inf(lo) && !is_inf(up) && lo > up) {
    if (lo > up + tol_of(d.cfg, up)) infeasible = true;
    else {
      lo = up;
      snapped = true;
    }
  }
  double k = d.row_out[i].v0;
  nu = P.side_src[2 * (int64_t)i + 1] == i ? d.rhs[i] : (is_inf(up) ? up : pos0(up + k));
  nl = snapped ? nu : (P.side_src[2 * (int64_t)i] == i ? d.lhs[i] : (is_inf(lo) ? lo : pos0(lo + k)));
  return nl != d.lhs[i] || nu != d.rhs[i];
}

__global__ void k_par_count(Dev d, ParScratch P) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  int k = 0;
  if (P.lead[i] >= 0) {
    k = 1;
    d.flags->merged = 1;
    if (d.K > 1) d.lpf[d.row_lp[i]].merged = 1;
  } else if (P.is_leader[i]) {
    double lo, up;
    bool inf;
    if (leader_sides(d, P, (int)i, lo, up, inf)) k = 1;
    if (inf) flag_infeasible(d, row_lp_of(d, (int)i));
    // a side that becomes finite locks the leader's columns (dual fixing):
    // listed in P.slot, which the pass no longer reads
    bool new_fin = (is_inf(d.lhs[i]) && !is_inf(lo)) || (is_inf(d.rhs[i]) && !is_inf(up));
    if (d.cfg.dual_fix && new_fin) P.slot[atomicAdd(&d.flags->lead_count, 1)] = (int)i;
  }
  d.cnt[i] = k;
}

// the listed leaders' new locks, before their sides are replaced: one
// wavefront per leader
__global__ void __launch_bounds__(PSL_BLOCK) k_par_locks(Dev d, ParScratch P) {
  int nl = d.flags->lead_count;
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int k = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); k < nl; k += wstride) {
    int i = P.slot[k];
    double lo, up;
    bool inf;
    leader_sides(d, P, i, lo, up, inf);
    unsigned long long lnew = is_inf(d.lhs[i]) && !is_inf(lo) ? 1ull : 0ull;
    unsigned long long rnew = is_inf(d.rhs[i]) && !is_inf(up) ? 1ull : 0ull;
    for (int p = d.rp[i] + lane_id(); p < d.rp[i + 1]; p += PSL_WAVE) {
      int j = d.ci[p];
      double2 b = d.bnd[j];
      if (b.x == b.y) continue;
      unsigned long long add = d.va[p] > 0 ? (lnew | (rnew << 32)) : (rnew | (lnew << 32));
      if (add) atomicAdd(&d.locks[j], add);
    }
  }
}

__global__ void k_par_emit(Dev d, ParScratch P, int64_t base, int round) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.m) return;
  int i = (int)t;
  Record r;
  r.side = 0;
  r.round = (uint16_t)round_of(d, row_lp_of(d, i), round);
  if (P.lead[i] >= 0) {
    int L = P.lead[i];
    r.type = REC_PARALLEL_ROW;
    r.i = i;
    r.j = -1;
    r.k = L;
    r.v[0] = P.lam[i];
    r.v[1] = d.lhs[i];
    r.v[2] = d.rhs[i];
    r.v[3] = 0.0;
    d.rec[base + d.off[t]] = r;
    d.row_on[i] = 0;
  } else if (P.is_leader[i]) {
    double lo, up;
    bool inf;
    if (!leader_sides(d, P, i, lo, up, inf)) return;
    r.type = REC_LEADER_SIDES;
    r.i = i;
    r.j = P.side_src[2 * (int64_t)i];
    r.k = P.side_src[2 * (int64_t)i + 1];
    r.v[0] = d.lhs[i];
    r.v[1] = d.rhs[i];
    r.v[2] = lo;
    r.v[3] = up;
    d.rec[base + d.off[t]] = r;
    d.lhs[i] = lo;
    d.rhs[i] = up;
  }
}

// ---------------------------------------------------------------------------
void launch_par_reset(const Dev& d, const ParScratch& p, hipStream_t s) {
  int64_t t = p.cap > d.m ? p.cap : d.m;
  int64_t blocks = (t + PSL_BLOCK - 1) / PSL_BLOCK;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_par_reset, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, p);
}

// column lengths lose the merged rows: one wavefront per listed row
__global__ void __launch_bounds__(PSL_BLOCK) k_par_drop(Dev d, ParScratch P) {
  int nv = d.flags->vlist_count;
  int wstride = gridDim.x * (PSL_BLOCK / PSL_WAVE);
  for (int k = blockIdx.x * (PSL_BLOCK / PSL_WAVE) + (threadIdx.x >> 6); k < nv; k += wstride) {
    int r = P.vlist[k];
    if (P.lead[r] < 0) continue;
    double lhs = d.lhs[r], rhs = d.rhs[r];  // a removed row is no leader: its own sides
    for (int p = d.rp[r] + lane_id(); p < d.rp[r + 1]; p += PSL_WAVE) {
      int j = d.ci[p];
      double2 b = d.bnd[j];
      if (b.x != b.y) drop_col(d, j, d.va[p], lhs, rhs);
    }
  }
}

__global__ void k_par_bits(Dev d, ParScratch P) {
  write_bits(P.abits, d.n, [&](int64_t j) {
    double2 b = d.bnd[j];
    return b.x != b.y;
  });
}

void launch_par_hash(const Dev& d, const ParScratch& p, const SweepGrid& g, hipStream_t s) {
  if (d.n > 0) {
    int64_t b = (d.n + PSL_BLOCK - 1) / PSL_BLOCK;
    if (b > 16384) b = 16384;
    hipLaunchKernelGGL(k_par_bits, dim3((unsigned)b), dim3(PSL_BLOCK), 0, s, d, p);
  }
  int total = 0;
  for (int b = 0; b < NBINS; ++b) total += g.nb[b];
  if (d.nlong > 0)
    hipLaunchKernelGGL(k_par_long_first, dim3((d.nlong + 3) / 4), dim3(PSL_BLOCK), 0, s, d, p);
  if (total > 0) hipLaunchKernelGGL(k_par_hash, dim3(total), dim3(PSL_BLOCK), 0, s, d, p, g);
  if (d.nlong > 0)
    hipLaunchKernelGGL(k_par_long_insert, dim3((d.nlong + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d, p);
  if (d.m > 0) hipLaunchKernelGGL(k_par_vlist, dim3((d.m + VLIST_BLOCK - 1) / VLIST_BLOCK), dim3(VLIST_BLOCK), 0, s, d, p);
}

void launch_par_drop(const Dev& d, const ParScratch& p, hipStream_t s) {
  hipLaunchKernelGGL(k_par_drop, dim3(1024), dim3(PSL_BLOCK), 0, s, d, p);
}

void launch_par_verify(const Dev& d, const ParScratch& p, hipStream_t s) {
  hipLaunchKernelGGL(k_par_verify, dim3(2048), dim3(PSL_BLOCK), 0, s, d, p);
  hipLaunchKernelGGL(k_par_src, dim3(1024), dim3(PSL_BLOCK), 0, s, d, p);
}

void launch_par_count(const Dev& d, const ParScratch& p, hipStream_t s) {
  if (d.m == 0) return;
  hipLaunchKernelGGL(k_par_count, dim3((d.m + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d, p);
  if (d.cfg.dual_fix) hipLaunchKernelGGL(k_par_locks, dim3(1024), dim3(PSL_BLOCK), 0, s, d, p);
}

void launch_par_emit(const Dev& d, const ParScratch& p, int64_t base, int round, hipStream_t s) {
  if (d.m == 0) return;
  hipLaunchKernelGGL(k_par_emit, dim3((d.m + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d, p, base, round);
}

}  // namespace psl
