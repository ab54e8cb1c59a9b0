// compact.hip -- emission of the reduced LP (section 3.3): kept rows x kept
// columns in their original order, sides shifted by the removed columns'
// constant contribution (canonical pairwise sum over the row, computed by the
// sweep in compaction mode), the removed columns' cost terms folded into the
// objective offset, and both the CSR and the transposed copy.
//
// Output positions come from exclusive scans of keep flags over the CSR
// positions and over the transposed copy's positions, so the kept entries keep
// their order in both layouts. In a batch the LPs are blocks of one LP, so
// each LP's kept rows, columns and entries are contiguous in these scans.
#include "bits.h"
#include "psl_kern.h"
#include "sweep.h"

namespace psl {

// kept rows and columns (as counts to scan, and the columns also as bytes
// for the position pass), the removed columns' cost terms
__global__ void k_cmp_flags(Dev d, CompactScratch c) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < d.m; i += stride) c.row_new[i] = d.row_on[i];
  for (int64_t j = t0; j < d.n; j += stride) {
    double2 b = d.bnd[j];
    bool kept = b.x != b.y;
    c.col_new[j] = kept;
    c.col_keep[j] = kept;
    c.terms[j] = kept ? 0.0 : pos0(d.c[j] * b.x);
  }
}

// the kept rows and columns as bits (L2-resident for the random lookups of
// the position and gather passes)
__global__ void k_cmp_bits(Dev d, CompactScratch c) {
  write_bits(c.rbits, d.m, [&](int64_t i) { return d.row_on[i] != 0; });
  write_bits(c.cbits, d.n, [&](int64_t j) { return c.col_keep[j] != 0; });
}

// kept positions of both layouts (a position is kept when its row and its
// column are): in CSR order the row is monotone and the column random, in
// the transposed copy the other way round; the random side reads bits
__global__ void k_cmp_pos_flags(Dev d, CompactScratch c) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= d.nnz; p += stride) {
    int ef = 0, qf = 0;
    if (p < d.nnz) {
      ef = d.row_on[c.rowid1[p + 1]] && bit_of(c.cbits, d.ci[p]);
      qf = bit_of(c.rbits, d.ri[p]) && c.col_keep[c.colid[p]];
    }
    c.eflag[p] = ef;
    c.qflag[p] = qf;
  }
}

// after the scans: the kept rows / columns before each bit word
__global__ void k_cmp_pre(Dev d, CompactScratch c) {
  int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (64 * w < d.m) c.rbits[w].pre = c.row_new[64 * w];
  if (64 * w < d.n) c.cbits[w].pre = c.col_new[64 * w];
}

__global__ void k_cmp_offset(const double* sum, double off, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = pos0(off + sum[0]);
}

// Batched presolve: each LP's reduced problem is numbered from 0 (its rows,
// columns and positions start at the LP's bases in c.lpr) and its row and
// column pointer arrays get one end entry each, at lpr.rb + k and lpr.cb + k.
__global__ void k_cmp_lpbase(Dev d, CompactScratch c, Reduced r) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > d.K) return;
  auto base = [&](int q) {
    int i0 = d.K > 1 ? d.lp_row0[q] : (q ? d.m : 0);
    int j0 = d.K > 1 ? d.lp_col0[q] : (q ? d.n : 0);
    LpRed b;
    b.rb = i0 < d.m ? c.row_new[i0] : c.totals[0];
    b.cb = j0 < d.n ? c.col_new[j0] : c.totals[1];
    b.eb = c.eflag[d.rp[i0]];
    b.qb = c.qflag[d.cp[j0]];
    return b;
  };
  LpRed b = base(k);
  c.lpr[k] = b;
  if (k < d.K) {
    LpRed e = base(k + 1);
    r.row_ptr[e.rb + k] = e.eb - b.eb;
    r.col_ptr[e.cb + k] = e.qb - b.qb;
  }
}

// kept entries of the CSR (new column ids from the column bits) ...
__global__ void k_cmp_gather_rows(Dev d, CompactScratch c, Reduced r) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < d.nnz; p += stride) {
    int pe = c.eflag[p];
    if (c.eflag[p + 1] != pe) {  // kept
      int j = d.ci[p];
      r.col_idx[pe] = rank_of(c.cbits, j) - (d.K > 1 ? c.lpr[d.col_lp[j]].cb : 0);
      r.val[pe] = d.va[p];
    }
  }
}

// ... and of the transposed copy (new row ids from the row bits)
__global__ void k_cmp_gather_cols(Dev d, CompactScratch c, Reduced r) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < d.nnz; p += stride) {
    int pq = c.qflag[p];
    if (c.qflag[p + 1] != pq) {
      int i = d.ri[p];
      r.row_idx[pq] = rank_of(c.rbits, i) - (d.K > 1 ? c.lpr[d.row_lp[i]].rb : 0);
      r.cval[pq] = d.cva[p];
    }
  }
}

__global__ void k_cmp_fill(Dev d, CompactScratch c, Reduced r) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = d.m, n = d.n;
  if (t < m) {
    int i = (int)t;
    if (!d.row_on[i]) return;
    int lp = row_lp_of(d, i);
    LpRed b = c.lpr[lp];
    int ri = c.row_new[i];
    double k = d.row_out[i].v0;  // constant of the removed columns
    double l = d.lhs[i], u = d.rhs[i];
    double nl = is_inf(l) ? l : pos0(l - k);
    double nu = is_inf(u) ? u : pos0(u - k);
    int p0 = c.eflag[d.rp[i]], p1 = c.eflag[d.rp[i + 1]];
    int len = p1 - p0;
    r.row_map[ri] = i - (d.K > 1 ? d.lp_row0[lp] : 0);
    r.lhs[ri] = nl;
    r.rhs[ri] = nu;
    r.row_ptr[ri + lp] = p0 - b.eb;
    r.row_class[ri] = len == 1 ? 1 : len == 2 ? (nl == nu ? 2 : 3) : 0;
    return;
  }
  if (t >= m + n) return;
  int j = (int)(t - m);
  double2 b = d.bnd[j];
  if (b.x == b.y) return;
  int lp = col_lp_of(d, j);
  LpRed cb = c.lpr[lp];
  int rj = c.col_new[j];
  int q0 = c.qflag[d.cp[j]], q1 = c.qflag[d.cp[j + 1]];
  int len = q1 - q0;
  r.col_map[rj] = j - (d.K > 1 ? d.lp_col0[lp] : 0);
  r.lb[rj] = b.x;
  r.ub[rj] = b.y;
  r.c[rj] = d.c[j];
  r.col_ptr[rj + lp] = q0 - cb.qb;
  bool fr = is_inf(b.x) && is_inf(b.y);
  r.col_class[rj] = len == 1 ? (fr ? 1 : 2) : len == 2 ? 3 : 0;
}

void compact_flags(const Dev& d, const CompactScratch& c, hipStream_t s) {
  int64_t t = d.nnz + 1;
  if (d.m > t) t = d.m;
  if (d.n > t) t = d.n;
  int64_t blocks = (t + PSL_BLOCK - 1) / PSL_BLOCK;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_cmp_flags, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, c);
  hipLaunchKernelGGL(k_cmp_bits, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, c);
  hipLaunchKernelGGL(k_cmp_pos_flags, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, c);
  scan_excl(c.row_new, c.row_new, d.m, c.totals + 0, c.ws, s);
  scan_excl(c.col_new, c.col_new, d.n, c.totals + 1, c.ws, s);
  int64_t words = (d.m > d.n ? d.m : d.n) / 64 + 1;
  hipLaunchKernelGGL(k_cmp_pre, dim3((unsigned)((words + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d, c);
  scan_excl(c.eflag, c.eflag, d.nnz + 1, c.totals + 2, c.ws, s);
  scan_excl(c.qflag, c.qflag, d.nnz + 1, c.totals + 3, c.ws, s);
}

void compact_write(const Dev& d, const CompactScratch& c, const Reduced& r, double obj_offset, hipStream_t s) {
  if (d.K == 1) {
    pairwise_sum(c.terms, d.n, c.pws, c.pws + 1, s);
    hipLaunchKernelGGL(k_cmp_offset, dim3(1), dim3(64), 0, s, (const double*)c.pws, obj_offset, c.offset);
  } else {
    segmented_pairwise_sum(c.terms, c.seg, c.seg_host, d.K, c.lp_off_in, c.offset, c.pws, s);
  }
  hipLaunchKernelGGL(k_cmp_lpbase, dim3((d.K + PSL_BLOCK) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d, c, r);
  if (d.nnz > 0) {
    int64_t blocks = (d.nnz + PSL_BLOCK - 1) / PSL_BLOCK;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_cmp_gather_rows, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, c, r);
    hipLaunchKernelGGL(k_cmp_gather_cols, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, c, r);
  }
  int64_t t = (int64_t)d.m + d.n;
  if (t < 1) t = 1;
  hipLaunchKernelGGL(k_cmp_fill, dim3((unsigned)((t + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d, c, r);
}

}  // namespace psl
