// ingest.hip -- validation, canonicalisation, the transposed copy of A, row
// binning and the input fixings ("round 0").
//
// The paper keeps A together with its transpose (section 3.2, "Internal data
// structures"). The transpose is built here by a stable radix sort of the CSR
// positions by column, so the rows of every column come out ascending.
#include "psl_kern.h"
#include "sweep.h"

namespace psl {

enum : int32_t {
  ERR_ROWPTR = 1, ERR_COLIDX = 2, ERR_COEF = 4, ERR_SIDE = 8, ERR_BOUND = 16, ERR_COST = 32
};

__device__ __forceinline__ void report(const Dev& d, int32_t bit, int64_t pos) {
  atomicOr(&d.flags->error, bit);
  atomicMin((long long*)&d.flags->error_pos, (long long)pos);
}

__device__ __forceinline__ double canon_inf(double v, double inf_value) {
  if (v >= inf_value) return __builtin_huge_val();
  if (v <= -inf_value) return -__builtin_huge_val();
  return pos0(v);
}

__global__ void k_check_rows(Dev d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  int32_t a = d.rp[i], b = d.rp[i + 1];
  if ((i == 0 && a != 0) || a < 0 || b < a || (int64_t)b > d.nnz || (i == d.m - 1 && (int64_t)b != d.nnz))
    report(d, ERR_ROWPTR, i);
  double l = d.lhs[i], r = d.rhs[i];
  double iv = d.cfg.inf_value;
  if (__builtin_isnan(l) || __builtin_isnan(r) || l >= iv || r <= -iv) report(d, ERR_SIDE, i);
  d.lhs[i] = canon_inf(l, iv);
  d.rhs[i] = canon_inf(r, iv);
}

__global__ void k_check_cols(Dev d, const double* lb_in, const double* ub_in, double* c_mut) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  double l = lb_in[j], u = ub_in[j], c = c_mut[j];
  double iv = d.cfg.inf_value;
  if (__builtin_isnan(l) || __builtin_isnan(u) || l >= iv || u <= -iv) report(d, ERR_BOUND, j);
  if (!__builtin_isfinite(c)) report(d, ERR_COST, j);
  d.bnd[j] = make_double2(canon_inf(l, iv), canon_inf(u, iv));
  c_mut[j] = pos0(c);
}

// rowid1[e] counts the rows ending at position e; its exclusive scan then
// gives, at index p + 1, the row holding CSR position p.
__global__ void k_row_ends(Dev d, int32_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  atomicAdd(&cnt[d.rp[i + 1]], 1);
}

__global__ void k_check_entries(Dev d, const int32_t* rowid1) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < d.nnz; p += (int64_t)gridDim.x * blockDim.x) {
    int row = rowid1[p + 1];
    int j = d.ci[p];
    if (j < 0 || j >= d.n || (p > d.rp[row] && d.ci[p - 1] >= j)) report(d, ERR_COLIDX, p);
    double a = d.va[p];
    if (!__builtin_isfinite(a) || a == 0.0) report(d, ERR_COEF, p);
  }
}

void launch_check_rows(const Dev& d, hipStream_t s) {
  if (d.m == 0) return;
  hipLaunchKernelGGL(k_check_rows, dim3((d.m + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d);
}

void check_cols(const Dev& d, const double* lb_in, const double* ub_in, double* c_mut, hipStream_t s) {
  if (d.n == 0) return;
  hipLaunchKernelGGL(k_check_cols, dim3((d.n + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d, lb_in, ub_in,
                     c_mut);
}

void build_rowid(const Dev& d, IngestScratch& sc, hipStream_t s) {
  fill_i32(sc.rowid1, 0, d.nnz + 1, s);
  if (d.m > 0)
    hipLaunchKernelGGL(k_row_ends, dim3((d.m + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d, sc.rowid1);
  scan_excl(sc.rowid1, sc.rowid1, d.nnz + 1, nullptr, sc.ws, s);
}

void launch_check_entries(const Dev& d, const int32_t* rowid1, hipStream_t s) {
  if (d.nnz == 0) return;
  int64_t blocks = (d.nnz + PSL_BLOCK - 1) / PSL_BLOCK;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_check_entries, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, rowid1);
}

// ---------------------------------------------------------------------------
// transposed copy
// ---------------------------------------------------------------------------
__global__ void k_csc_gather(Dev d, const int32_t* perm, const int32_t* rowid1, int32_t* ri, double* cva) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < d.nnz; q += (int64_t)gridDim.x * blockDim.x) {
    int p = perm ? perm[q] : (int)q;
    ri[q] = rowid1[p + 1];
    cva[q] = d.va[p];
  }
}

// cp from the column-sorted keys: position q starts every column in
// (keys[q-1], keys[q]] (keys[-1] = -1, keys[nnz] = n), so empty columns get
// the next column's start
__global__ void k_col_ptr(Dev d, const uint32_t* keys, int32_t* cp) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= d.nnz; q += (int64_t)gridDim.x * blockDim.x) {
    int64_t prev = q > 0 ? (int64_t)keys[q - 1] : -1;
    int64_t cur = q < d.nnz ? (int64_t)keys[q] : (int64_t)d.n;
    // keys were validated (< n); clamped all the same so no store leaves cp
    prev = prev < (int64_t)d.n ? prev : (int64_t)d.n;
    cur = cur < (int64_t)d.n ? cur : (int64_t)d.n;
    for (int64_t j = prev + 1; j <= cur; ++j) cp[j] = (int32_t)q;
  }
}

__global__ void k_col_len(Dev d, const int32_t* cp, int32_t* col_len) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  col_len[j] = cp[j + 1] - cp[j];
}

// Stable transpose by LSD radix passes over the column index (at most 8 bits
// a pass, the bits split evenly), moving row and value with each key; the
// last pass writes the transposed copy itself. vtmp: nnz doubles of scratch.
// Returns the column of every position of the transposed copy (the sorted
// keys), which compaction uses.
const uint32_t* build_csc(const Dev& d, int32_t* cp, int32_t* ri, double* cva, int32_t* col_len, IngestScratch& sc,
                          double* vtmp, hipStream_t s) {
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < (int64_t)d.n) ++bits;
  int passes = (bits + 7) / 8;
  const uint32_t* kin = (const uint32_t*)d.ci;
  if (passes == 0) {
    // at most one column: the transposed copy is the CSR order
    if (d.nnz > 0) {
      int64_t blocks = (d.nnz + PSL_BLOCK - 1) / PSL_BLOCK;
      if (blocks > 16384) blocks = 16384;
      hipLaunchKernelGGL(k_csc_gather, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)nullptr,
                         sc.rowid1, ri, cva);
    }
  } else {
    int per = (bits + passes - 1) / passes;
    const int32_t* rin = nullptr;
    const double* vin = d.va;
    uint32_t* kb[2] = {sc.k0, sc.k1};
    int32_t* rb[2] = {sc.v0, sc.v1};
    for (int pass = 0, shift = 0; pass < passes; ++pass, shift += per) {
      int b = bits - shift < per ? bits - shift : per;
      bool last = pass == passes - 1;
      // the values end in cva after an odd number of hops from it
      double* vout = ((passes - 1 - pass) % 2 == 0) ? cva : vtmp;
      int32_t* rout = last ? ri : rb[pass & 1];
      uint32_t* kout = kb[pass & 1];
      radix_pass_payload(kin, rin, sc.rowid1, vin, kout, rout, vout, d.nnz, shift, b, sc.ws, s);
      kin = kout;
      rin = rout;
      vin = vout;
    }
  }
  {
    int64_t blocks = (d.nnz + 1 + PSL_BLOCK - 1) / PSL_BLOCK;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_col_ptr, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, kin, cp);
  }
  if (d.n > 0)
    hipLaunchKernelGGL(k_col_len, dim3((d.n + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d,
                       (const int32_t*)cp, col_len);
  return kin;
}

// ---------------------------------------------------------------------------
// row bins by CSR length, and the chunk table of long rows
// ---------------------------------------------------------------------------
// bin of every row, and the bin sizes (counted per wavefront by ballots, per
// workgroup in LDS, then one global add per workgroup and bin)
__global__ void k_bin_keys(Dev d, int32_t t_long, int32_t t_g8, uint32_t* keys, int32_t* counts) {
  __shared__ int c[NBINS];
  if (threadIdx.x < NBINS) c[threadIdx.x] = 0;
  __syncthreads();
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < d.m; i0 += stride) {
    int64_t i = i0 + threadIdx.x;
    int b = -1;
    if (i < d.m) {
      int len = d.rp[i + 1] - d.rp[i];
      b = len <= 4 ? BIN_G4 : len <= t_g8 ? BIN_G8 : len <= 16 ? BIN_G16 : len > t_long ? BIN_LONG
        : len <= 64 ? BIN_W1 : len <= 256 ? BIN_W4 : BIN_W8;
      keys[i] = (uint32_t)b;
    }
#pragma unroll
    for (int k = 0; k < NBINS; ++k) {
      int cnt = __popcll(__ballot(b == k));
      if (lane_id() == 0 && cnt) atomicAdd(&c[k], cnt);
    }
  }
  __syncthreads();
  if (threadIdx.x < NBINS && c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], c[threadIdx.x]);
}

__global__ void k_bin_fill(Dev d, const int32_t* rows, BinEnt* bins) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.m) return;
  int row = rows[k];
  int a = d.rp[row], b = d.rp[row + 1];
  bins[k] = BinEnt{row, a, b - a, 0};
}

void build_bins(const Dev& d, const int32_t* thresholds, BinEnt* bins, int32_t* counts, IngestScratch& sc,
                hipStream_t s) {
  fill_i32(counts, 0, NBINS, s);
  if (d.m == 0) return;
  unsigned blocks = (unsigned)((d.m + PSL_BLOCK - 1) / PSL_BLOCK);
  unsigned kb = blocks < 1024 ? blocks : 1024;
  hipLaunchKernelGGL(k_bin_keys, dim3(kb), dim3(PSL_BLOCK), 0, s, d, thresholds[0], thresholds[2], sc.k0, counts);
  radix_pass(sc.k0, nullptr, sc.k1, sc.v0, d.m, 0, 3, sc.ws, s);
  hipLaunchKernelGGL(k_bin_fill, dim3(blocks), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)sc.v0, bins);
}

// ---------------------------------------------------------------------------
// filtering of the bin lists and the chunk list down to the active rows
// ---------------------------------------------------------------------------
// passes per chunk: the requested size, doubled until the row has at most
// LONG_MAX_CHUNKS chunks (chunk sizes stay powers of two times PASS_LEN)
__global__ void k_long_count(Dev d, int npass0, int32_t* cnt, int32_t* cnt2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.nlong) return;
  BinEnt be = d.bins[d.bin_off[BIN_LONG] + k];
  int row = be.row;
  int64_t len = be.len;
  int64_t np = npass0;
  while ((len + np * PASS_LEN - 1) / (np * PASS_LEN) > LONG_MAX_CHUNKS) np *= 2;
  if (np > LONG_MAX_PASSES) {
    atomicOr(&d.flags->error, 64);  // row too long for the chunk table
    np = LONG_MAX_PASSES;
  }
  int nch = (int)((len + np * PASS_LEN - 1) / (np * PASS_LEN));
  d.lrow[k] = LongRow{row, 0, nch, (int32_t)np};
  cnt[k] = nch;
  cnt2[k] = 2 * (int)len;  // candidate entries of the row's chunks
}

__global__ void k_long_fill(Dev d, const int32_t* off, const int32_t* uoff, LongChunk* chunks) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.nlong) return;
  LongRow lr = d.lrow[k];
  lr.chunk0 = off[k];
  d.lrow[k] = lr;
  for (int c = 0; c < lr.nchunk; ++c)
    chunks[lr.chunk0 + c] = LongChunk{lr.row, c * lr.npass * PASS_LEN, k, lr.npass,
                                      uoff[k] + 2 * c * lr.npass * PASS_LEN, lr.chunk0 + c};
}

void build_long_chunks(const Dev& d, int npass0, LongChunk* chunks, int32_t* cnt, int32_t* cnt2, int32_t* totals,
                       int32_t* ws, hipStream_t s) {
  if (d.nlong == 0) {
    fill_i32(totals, 0, 2, s);
    return;
  }
  unsigned blocks = (unsigned)((d.nlong + PSL_BLOCK - 1) / PSL_BLOCK);
  hipLaunchKernelGGL(k_long_count, dim3(blocks), dim3(PSL_BLOCK), 0, s, d, npass0, cnt, cnt2);
  scan_excl(cnt, cnt, d.nlong, totals, ws, s);
  scan_excl(cnt2, cnt2, d.nlong, totals + 1, ws, s);
  hipLaunchKernelGGL(k_long_fill, dim3(blocks), dim3(PSL_BLOCK), 0, s, d, (const int32_t*)cnt, (const int32_t*)cnt2,
                     chunks);
}

struct BinOffsets {
  int32_t off[NBINS + 1];
};

// The filter works in tiles of RB_TILE items (RB_ITEMS per thread, striped so
// the loads coalesce): the entry tiles of the bin list, then the tiles of the
// chunk list. A first launch takes the keep decisions (one byte per item) and
// counts each tile's kept items, a scan of the tile counts gives each tile's
// output offset, and a second launch writes the kept items in input order.
// The decisions are taken once: the second launch clears dirty flags, which
// the chunks of a long row would otherwise read after its entry cleared them.
#define RB_ITEMS 4
#define RB_TILE (PSL_BLOCK * RB_ITEMS)

size_t rebin_flag_bytes(int64_t nent, int64_t nch) { return (size_t)(nent + nch + 2 * RB_TILE); }

struct RebinArgs {
  const BinEnt* bins;
  int32_t nent;
  const LongChunk* chunks;
  int32_t nch;
  uint8_t* dirty;        // dirty flags (used when the mode asks for them)
  int use_dirty, inert;  // filter mode, unless mode != nullptr
  const int32_t* mode;   // device: bit 0 = dirty rows only, bit 1 = skip inert rows
  uint8_t* keep;         // [T * RB_TILE] keep decisions
};

__device__ __forceinline__ void rebin_mode(const RebinArgs& a, const uint8_t*& dirty, bool& inert) {
  int md = a.mode ? *a.mode : ((a.use_dirty ? 1 : 0) | (a.inert ? 2 : 0));
  dirty = (md & 1) ? a.dirty : nullptr;
  inert = (md & 2) != 0;
}

// keep a bin entry (and the chunks of a long row) when its row is active, its
// LP still presolving, with a dirty array touched by a column change since it
// was last swept, and with inert set not inert; no short-circuit loads, so the
// loads of a thread's items are in flight together
__device__ __forceinline__ bool keep_row_flat(const Dev& d, int row, const uint8_t* dirty, bool inert) {
  bool on = d.row_on[row] != 0;
  bool dt = dirty ? dirty[row] != 0 : true;
  bool lp = d.K == 1 ? true : d.lp_ok[d.row_lp[row]] != 0;
  bool live = true;
  if (inert) live = !row_inert(d.rinf[row], d.lhs[row], d.rhs[row]);
  return on && dt && lp && live;
}

__global__ void __launch_bounds__(PSL_BLOCK) k_rebin_count(Dev d, RebinArgs a, int te, int T, int32_t* tile_sum,
                                                           int32_t* totals) {
  int c = 0;
  int tile = blockIdx.x;
  if (tile < T) {
    const uint8_t* dirty;
    bool inert;
    rebin_mode(a, dirty, inert);
    bool ct = tile >= te;
    int64_t base = (int64_t)(ct ? tile - te : tile) * RB_TILE + threadIdx.x;
    int64_t lim = ct ? a.nch : a.nent;
    int rows[RB_ITEMS];
#pragma unroll
    for (int k = 0; k < RB_ITEMS; ++k) {
      int64_t idx = base + (int64_t)k * PSL_BLOCK;
      rows[k] = idx < lim ? (ct ? a.chunks[idx].row : a.bins[idx].row) : -1;
    }
#pragma unroll
    for (int k = 0; k < RB_ITEMS; ++k) {
      bool f = keep_row_flat(d, rows[k] >= 0 ? rows[k] : 0, dirty, inert) & (rows[k] >= 0);
      a.keep[(int64_t)tile * RB_TILE + k * PSL_BLOCK + threadIdx.x] = f ? 1 : 0;
      c += f;
    }
  }
  int tot;
  block_excl_scan(c, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    tile_sum[T] = 0;
    totals[1] = 0;  // kept nonzeros, summed by the scatter
  }
}

// tile_off: exclusive scan of the tile counts (T + 1 entries)
__global__ void __launch_bounds__(PSL_BLOCK) k_rebin_scatter(RebinArgs a, int te, int T, const int32_t* tile_off,
                                                             BinEnt* out, LongChunk* cout, BinOffsets old,
                                                             int32_t* new_off, int32_t* totals) {
  __shared__ int wcnt[RB_ITEMS][PSL_BLOCK / PSL_WAVE];
  int w = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    totals[0] = tile_off[te];
    totals[2] = tile_off[T] - tile_off[te];
  }
  if (blockIdx.x == 0 && threadIdx.x <= NBINS && old.off[threadIdx.x] == a.nent)
    new_off[threadIdx.x] = tile_off[te];
  int tile = blockIdx.x;
  if (tile >= T) return;
  bool ct = tile >= te;
  int64_t base_idx = (int64_t)(ct ? tile - te : tile) * RB_TILE + threadIdx.x;
  bool f[RB_ITEMS];
  int pre[RB_ITEMS];
#pragma unroll
  for (int k = 0; k < RB_ITEMS; ++k) {
    f[k] = a.keep[(int64_t)tile * RB_TILE + k * PSL_BLOCK + threadIdx.x] != 0;
    unsigned long long bal = __ballot(f[k]);
    pre[k] = __popcll(bal & lanemask_lt());
    if (lane_id() == 0) wcnt[k][w] = __popcll(bal);
  }
  __syncthreads();
  // exclusive prefix of item (k, thread) in index order (k-major)
  int run = 0;
#pragma unroll
  for (int k = 0; k < RB_ITEMS; ++k) {
    int row_tot = 0, before = 0;
#pragma unroll
    for (int v = 0; v < PSL_BLOCK / PSL_WAVE; ++v) {
      int c = wcnt[k][v];
      row_tot += c;
      if (v < w) before += c;
    }
    pre[k] += run + before;
    run += row_tot;
  }
  int64_t base = (int64_t)tile_off[tile] - (ct ? tile_off[te] : 0);
  const uint8_t* dirty;
  bool inert;
  rebin_mode(a, dirty, inert);
  int len = 0;
#pragma unroll
  for (int k = 0; k < RB_ITEMS; ++k) {
    int64_t idx = base_idx + (int64_t)k * PSL_BLOCK;
    int64_t pos = base + pre[k];
    if (!ct) {
      if (idx < a.nent) {
#pragma unroll
        for (int b = 0; b <= NBINS; ++b)
          if (old.off[b] == idx) new_off[b] = (int32_t)pos;
      }
      if (f[k]) {
        BinEnt be = a.bins[idx];
        out[pos] = be;
        len += be.len;
        if (dirty) a.dirty[be.row] = 0;  // swept now
      }
    } else if (f[k]) {
      cout[pos] = a.chunks[idx];
    }
  }
  int tot;
  block_excl_scan(len, &tot);
  if (tot && threadIdx.x == 0) atomicAdd(&totals[1], tot);
}

void rebin(const Dev& d, const BinEnt* bins_in, const int32_t* off_in, const LongChunk* chunks_in, int32_t nch,
           BinEnt* bins_out, LongChunk* chunks_out, uint8_t* dirty, bool inert, const int32_t* mode,
           uint8_t* keep, int32_t* tile_sum, int32_t* new_off, int32_t* totals, int32_t* ws, hipStream_t s) {
  BinOffsets bo;
  for (int b = 0; b <= NBINS; ++b) bo.off[b] = off_in[b];
  RebinArgs a;
  a.bins = bins_in;
  a.nent = off_in[NBINS];
  a.chunks = chunks_in;
  a.nch = nch;
  a.dirty = mode ? d.dirty : dirty;
  a.use_dirty = dirty != nullptr;
  a.inert = inert ? 1 : 0;
  a.mode = mode;
  a.keep = keep;
  int te = (int)(((int64_t)a.nent + RB_TILE - 1) / RB_TILE);
  int tc = (int)(((int64_t)nch + RB_TILE - 1) / RB_TILE);
  int T = te + tc;
  unsigned grid = (unsigned)(T > 0 ? T : 1);
  hipLaunchKernelGGL(k_rebin_count, dim3(grid), dim3(PSL_BLOCK), 0, s, d, a, te, T, tile_sum, totals);
  scan_excl(tile_sum, tile_sum, (int64_t)T + 1, nullptr, ws, s);
  hipLaunchKernelGGL(k_rebin_scatter, dim3(grid), dim3(PSL_BLOCK), 0, s, a, te, T, (const int32_t*)tile_sum,
                     bins_out, chunks_out, bo, new_off, totals);
}

// Rows of the columns whose bounds changed (or that were fixed) this round,
// from the transposed copy; their infinite-contribution counts follow the
// bounds that became finite. One wavefront per 64 columns walks the entries of
// its changed columns; columns of more than MARK_DENSE entries (listed once
// at ingest) are walked by every workgroup of a second launch.
#define MARK_DENSE 4096
#define MARK_MASK (CC_LB | CC_UB | CC_FIX)

// One entry (q, row i) of a changed column: mark the row (when the next
// round sweeps dirty rows only), and (with count) lower its infinite-
// contribution counts when the column's lb / ub became finite.
__device__ __forceinline__ void mark_entry(const Dev& d, int64_t q, int code, bool mark, bool count) {
  int i = d.ri[q];
  if (mark) d.dirty[i] = 1;
  if (count && (code & (CC_LBFIN | CC_UBFIN))) {
    bool pos = d.cva[q] > 0;
    bool lbf = (code & CC_LBFIN) != 0, ubf = (code & CC_UBFIN) != 0;
    if ((lbf && pos) || (ubf && !pos)) atomicSub(&d.rinf[i].x, 1);  // min contribution now finite
    if ((lbf && !pos) || (ubf && pos)) atomicSub(&d.rinf[i].y, 1);  // max contribution now finite
  }
}

// columns the marking pass walks: changed ones when rows are marked, those
// with a bound that became finite when counts are kept
__device__ __forceinline__ bool mark_col(int code, int mode) {
  return ((mode & 1) && (code & MARK_MASK)) || ((mode & 2) && (code & (CC_LBFIN | CC_UBFIN)));
}

// The next round's selection mode from this round's totals (bit 0: sweep only
// the rows touched by a change, when few columns changed and allow is set;
// bit 1: keep the infinite-contribution counts, when few bounds became finite)
struct RoundMode {
  int allow, incr_factor, count_factor;
};

__device__ __forceinline__ int round_mode(const Dev& d, const RoundMode& rm) {
  int64_t changed = (int64_t)d.flags->round_total - d.flags->rows_removed;
  bool incr = rm.allow && changed * rm.incr_factor < (int64_t)d.n;
  bool counts = (int64_t)d.flags->fin_cols * rm.count_factor < (int64_t)d.n;
  return (incr ? 1 : 0) | (counts ? 2 : 0);
}

__global__ void __launch_bounds__(PSL_BLOCK) k_mark_sparse(Dev d, RoundMode rm) {
  int mode = round_mode(d, rm);
  if (blockIdx.x == 0 && threadIdx.x == 0) d.flags->mode = mode;
  if (mode == 0) return;
  int64_t j = (int64_t)blockIdx.x * PSL_BLOCK + threadIdx.x;
  bool ch = false;
  int q0 = 0, q1 = 0, code = 0;
  if (j < d.n) code = d.col_code[j];
  if (mark_col(code, mode)) {
    q0 = d.cp[j];
    q1 = d.cp[j + 1];
    ch = q1 - q0 <= MARK_DENSE;
  }
  unsigned long long mask = __ballot(ch);
  int lane = lane_id();
  while (mask) {
    int l = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    int a = __shfl(q0, l, PSL_WAVE), b = __shfl(q1, l, PSL_WAVE), cl = __shfl(code, l, PSL_WAVE);
    for (int q = a + lane; q < b; q += PSL_WAVE) mark_entry(d, q, cl, mode & 1, mode & 2);
  }
}

// every workgroup lists the changed dense columns (in slices of 1024, checked
// in parallel) and walks a grid-strided share of their entries
__global__ void __launch_bounds__(PSL_BLOCK) k_mark_dense(Dev d, RoundMode rm) {
  __shared__ int32_t list[1024];
  __shared__ int32_t cnt;
  int mode = round_mode(d, rm);
  if (mode == 0) return;
  int nd = *d.n_dense;
  for (int k0 = 0; k0 < nd; k0 += 1024) {
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int k = k0 + threadIdx.x; k < nd && k < k0 + 1024; k += PSL_BLOCK) {
      int j = d.dense_cols[k];
      if (mark_col(d.col_code[j], mode)) list[atomicAdd(&cnt, 1)] = j;
    }
    __syncthreads();
    int nc = cnt;
    for (int c = 0; c < nc; ++c) {
      int j = list[c];
      int code = d.col_code[j];
      int64_t q1 = d.cp[j + 1];
      for (int64_t q = d.cp[j] + (int64_t)blockIdx.x * PSL_BLOCK + threadIdx.x; q < q1;
           q += (int64_t)gridDim.x * PSL_BLOCK)
        mark_entry(d, q, code, mode & 1, mode & 2);
    }
    __syncthreads();
  }
}

// the columns of more than MARK_DENSE entries (order irrelevant)
__global__ void k_dense_cols(Dev d) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  if (d.cp[j + 1] - d.cp[j] > MARK_DENSE) d.dense_cols[atomicAdd(d.n_dense, 1)] = (int32_t)j;
}

void list_dense_cols(const Dev& d, hipStream_t s) {
  fill_i32(d.n_dense, 0, 1, s);
  if (d.n > 0)
    hipLaunchKernelGGL(k_dense_cols, dim3((unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d);
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void mark_dirty(const Dev& d, bool clear_first, bool allow_incremental, int incr_factor, int count_factor,
                hipStream_t s) {
  if (clear_first && d.m > 0) {
    int64_t b = (d.m + PSL_BLOCK - 1) / PSL_BLOCK;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)(b > 4096 ? 4096 : b)), dim3(PSL_BLOCK), 0, s, d.dirty, (uint8_t)0,
                       (int64_t)d.m);
  }
  RoundMode rm{allow_incremental ? 1 : 0, incr_factor, count_factor};
  unsigned blocks = (unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK);
  hipLaunchKernelGGL(k_mark_sparse, dim3(blocks > 0 ? blocks : 1), dim3(PSL_BLOCK), 0, s, d, rm);
  if (d.nnz > 0 && d.n > 0) hipLaunchKernelGGL(k_mark_dense, dim3(1024), dim3(PSL_BLOCK), 0, s, d, rm);
}

// ---------------------------------------------------------------------------
// state initialisation and round 0 (input fixings, crossed bounds / sides)
// ---------------------------------------------------------------------------
__global__ void k_init_state(Dev d) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < d.m) {
    d.row_on[t] = 1;
    d.row_code[t] = RC_KEEP;
  }
  if (t < d.n) {
    double2 b = d.bnd[t];
    d.touch[t] = 1;  // the first round decides every column
    d.bkey[2 * t] = dkey(b.x);
    d.bkey[2 * t + 1] = dkey(b.y);
    d.src[2 * t] = 0x7FFFFFFF;
    d.src[2 * t + 1] = 0x7FFFFFFF;
    d.col_code[t] = 0;
  }
  if (t == 0) {
    Flags f;
    f.infeasible = f.unbounded = f.error = f.merged = 0;
    f.cand_count = f.round_total = f.vlist_count = f.rows_removed = 0;
    f.fin_cols = f.mode = 0;
    f.error_pos = 0x7FFFFFFFFFFFFFFFLL;
    *d.flags = f;
  }
}

void launch_init_state(const Dev& d, hipStream_t s) {
  int64_t t = d.m > d.n ? d.m : d.n;
  if (t < 1) t = 1;
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)((t + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d);
}

__global__ void k_round0_count(Dev d) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = d.m, n = d.n;
  if (t < m) {
    d.cnt[t] = 0;
    double l = d.lhs[t], r = d.rhs[t];
    if (!is_inf(l) && !is_inf(r) && l > r + tol_of(d.cfg, r)) flag_infeasible(d, row_lp_of(d, (int)t));
    return;
  }
  if (t >= m + n) return;
  int j = (int)(t - m);
  double2 b = d.bnd[j];
  int k = 0;
  if (!is_inf(b.x) && !is_inf(b.y)) {
    if (b.x > b.y + tol_of(d.cfg, b.y)) flag_infeasible(d, col_lp_of(d, j));
    if (b.y - b.x <= d.cfg.fix_tol * mx1(b.x)) k = 1;
  }
  d.cnt[t] = k;
}

__global__ void k_round0_emit(Dev d, int64_t base) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = d.m, n = d.n;
  if (t < m || t >= m + n) return;
  int j = (int)(t - m);
  double2 b = d.bnd[j];
  if (is_inf(b.x) || is_inf(b.y) || !(b.y - b.x <= d.cfg.fix_tol * mx1(b.x))) return;
  Record r;
  r.type = REC_FIX_COL;
  r.side = 0;
  r.round = 0;
  r.i = -1;
  r.j = j;
  r.k = -1;
  r.v[0] = b.x;
  r.v[1] = d.c[j];
  r.v[2] = 0.0;
  r.v[3] = 0.0;
  d.rec[base + d.off[t]] = r;
  d.bnd[j] = make_double2(b.x, b.x);
  d.bkey[2 * (int64_t)j + 1] = dkey(b.x);
}

void launch_round0_count(const Dev& d, hipStream_t s) {
  int64_t t = (int64_t)d.m + d.n;
  if (t == 0) return;
  hipLaunchKernelGGL(k_round0_count, dim3((unsigned)((t + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d);
}

void launch_round0_emit(const Dev& d, int64_t base, hipStream_t s) {
  int64_t t = (int64_t)d.m + d.n;
  if (t == 0) return;
  hipLaunchKernelGGL(k_round0_emit, dim3((unsigned)((t + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d,
                     base);
}

}  // namespace psl
