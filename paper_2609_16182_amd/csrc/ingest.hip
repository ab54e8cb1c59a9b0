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
// the next column's start. A thread writes at most the last COLPTR_RUN
// entries of its run (always cp[keys[q]], the start of a nonempty column, and
// cp[n]); longer runs of empty columns, e.g. a block of columns that appear in
// no row, are left at -1 (cp is filled with -1 before) and resolved per column
// in k_col_len, so no thread loops over a long run.
#define COLPTR_RUN 64
__global__ void k_col_ptr(Dev d, const uint32_t* keys, int32_t* cp) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= d.nnz; q += (int64_t)gridDim.x * blockDim.x) {
    int64_t prev = q > 0 ? (int64_t)keys[q - 1] : -1;
    int64_t cur = q < d.nnz ? (int64_t)keys[q] : (int64_t)d.n;
    // keys were validated (< n); clamped all the same so no store leaves cp
    prev = prev < (int64_t)d.n ? prev : (int64_t)d.n;
    cur = cur < (int64_t)d.n ? cur : (int64_t)d.n;
    int64_t j0 = cur - prev > COLPTR_RUN ? cur - COLPTR_RUN : prev;
    for (int64_t j = j0 + 1; j <= cur; ++j) cp[j] = (int32_t)q;
  }
}

// first position whose key is >= j (keys ascend): the start of column j
__device__ __forceinline__ int32_t col_start(const uint32_t* keys, int64_t nnz, int64_t j) {
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return (int32_t)lo;
}

// column lengths; entries of cp a long run left at -1 get the start of the
// next nonempty column by a search over the keys (cp[n] is always written)
__global__ void k_col_len(Dev d, const uint32_t* keys, int32_t* cp, int32_t* col_len) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  int32_t a = cp[j], b = cp[j + 1];
  if (a < 0) {
    a = col_start(keys, d.nnz, j);
    cp[j] = a;
  }
  if (b < 0) b = col_start(keys, d.nnz, j + 1);  // written by thread j + 1
  col_len[j] = b - a;
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
  fill_i32(cp, -1, d.n + 1, s);
  {
    int64_t blocks = (d.nnz + 1 + PSL_BLOCK - 1) / PSL_BLOCK;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_col_ptr, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, kin, cp);
  }
  if (d.n > 0)
    hipLaunchKernelGGL(k_col_len, dim3((d.n + PSL_BLOCK - 1) / PSL_BLOCK), dim3(PSL_BLOCK), 0, s, d, kin, cp,
                       col_len);
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

// ---------------------------------------------------------------------------
// row selection: the rows a round sweeps, as bin lists and long-row chunks
// ---------------------------------------------------------------------------
// A pass over all rows in tiles of SEL_TILE (SEL_ITEMS a thread, striped so
// the loads coalesce): a first launch takes each row's decision (one byte:
// 0, or 1 + its bin) and counts, per tile, the kept rows of every bin, the
// chunks of the kept long rows and the kept nonzeros; one scan of the counts
// (bin-major) gives every tile its output offsets; a second launch writes the
// kept rows in row order into contiguous bins and copies the kept long rows'
// chunks from the ingest chunk table. The row data of a row is read only
// when its cheap tests (active; marked, when only marked rows are wanted)
// pass, so a selection of few marked rows reads about a byte per row.
#define SEL_ITEMS 4
#define SEL_TILE (PSL_BLOCK * SEL_ITEMS)
static_assert(SEL_TILE == 1024, "a selection tile is a tile of the marks");
#define SEL_COUNTS (NBINS + 2)  // rows per bin, long-row chunks, nonzeros

size_t select_keep_bytes(int64_t m) { return (size_t)(m + 2 * SEL_TILE); }
size_t select_count_ints(int64_t m) { return (size_t)(SEL_COUNTS * ((m + SEL_TILE - 1) / SEL_TILE + 1) + 2); }

struct SelArgs {
  const int32_t* mode_dev;  // the device's mode (bit 0: marked rows only; bit 1:
  int mode_host;            // inert rows skipped), or mode_host without one
  int t_long, t_g8;         // bin thresholds of the ingest
  uint8_t* keep;            // per row: 0, or 1 + its bin
  int32_t* cnt;             // SEL_COUNTS * T + 1 counts, scanned in place
};

// bin of a row of len entries (the bins of the ingest)
__device__ __forceinline__ int bin_of_len(int len, int t_long, int t_g8) {
  return len <= 4 ? BIN_G4 : len <= t_g8 ? BIN_G8 : len <= 16 ? BIN_G16 : len > t_long ? BIN_LONG
       : len <= 64 ? BIN_W1 : len <= 256 ? BIN_W4 : BIN_W8;
}

// index of long row `row` in d.lrow (ascending rows; the row is long)
__device__ __forceinline__ int long_row_index(const Dev& d, int row) {
  int lo = 0, hi = d.nlong - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (d.lrow[mid].row < row) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int sel_mode(const SelArgs& a) { return a.mode_dev ? *a.mode_dev : a.mode_host; }

__global__ void __launch_bounds__(PSL_BLOCK) k_sel_count(Dev d, SelArgs a, int T) {
  __shared__ int red[PSL_BLOCK / PSL_WAVE][SEL_COUNTS];
  int tile = blockIdx.x;
  int mode = sel_mode(a);
  int c[SEL_COUNTS];
#pragma unroll
  for (int j = 0; j < SEL_COUNTS; ++j) c[j] = 0;
  // marked rows only: a tile without a mark keeps nothing (its keep bytes
  // are not read)
  if ((mode & 1) && tile < T && !d.dirty_tile[tile]) {
    if (threadIdx.x < SEL_COUNTS) a.cnt[(int64_t)threadIdx.x * T + tile] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[(int64_t)SEL_COUNTS * T] = 0;
    return;
  }
  if (tile < T) {
    // level by level for all items, without branches around the loads (a
    // row that fails the cheap tests reads row 0's data, which is cached)
    int64_t i[SEL_ITEMS];
    bool cand[SEL_ITEMS];
#pragma unroll
    for (int k = 0; k < SEL_ITEMS; ++k) {
      i[k] = (int64_t)tile * SEL_TILE + k * PSL_BLOCK + threadIdx.x;
      int64_t ii = i[k] < d.m ? i[k] : 0;
      uint8_t on = d.row_on[ii], dt = d.dirty[ii];
      cand[k] = i[k] < d.m && on != 0 && (!(mode & 1) || dt != 0);
    }
    int r0[SEL_ITEMS], r1[SEL_ITEMS], lpi[SEL_ITEMS];
    int2 rf[SEL_ITEMS];
    double lh[SEL_ITEMS], rh[SEL_ITEMS];
#pragma unroll
    for (int k = 0; k < SEL_ITEMS; ++k) {
      int64_t jj = cand[k] ? i[k] : 0;
      r0[k] = d.rp[jj];
      r1[k] = d.rp[jj + 1];
      lpi[k] = d.K > 1 ? d.row_lp[jj] : 0;
      if (mode & 2) {
        rf[k] = d.rinf[jj];
        lh[k] = d.lhs[jj];
        rh[k] = d.rhs[jj];
      }
    }
#pragma unroll
    for (int k = 0; k < SEL_ITEMS; ++k) {
      bool keep = cand[k];
      if (d.K > 1) keep = keep && d.lp_ok[lpi[k]] != 0;
      if (mode & 2) keep = keep && !row_inert(rf[k], lh[k], rh[k]);
      uint8_t kb = 0;
      if (keep) {
        int len = r1[k] - r0[k];
        int bin = bin_of_len(len, a.t_long, a.t_g8);
        kb = (uint8_t)(1 + bin);
#pragma unroll
        for (int b = 0; b < NBINS; ++b) c[b] += bin == b;
        if (bin == BIN_LONG) c[NBINS] += d.lrow[long_row_index(d, (int)i[k])].nchunk;
        c[NBINS + 1] += len;
      }
      a.keep[(int64_t)tile * SEL_TILE + k * PSL_BLOCK + threadIdx.x] = kb;
    }
  }
  int w = threadIdx.x >> 6;
  // a tile without kept rows (most tiles of a round that sweeps few marked
  // rows) writes zeros without the reductions
  if (!__syncthreads_or(c[NBINS + 1] != 0 || c[BIN_G4] + c[BIN_G8] + c[BIN_G16] + c[BIN_W1] + c[BIN_W4] + c[BIN_W8] +
                                                    c[BIN_LONG] != 0)) {
    if (threadIdx.x < SEL_COUNTS && tile < T) a.cnt[(int64_t)threadIdx.x * T + tile] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[(int64_t)SEL_COUNTS * T] = 0;
    return;
  }
#pragma unroll
  for (int j = 0; j < SEL_COUNTS; ++j) {
    int x = c[j];
#pragma unroll
    for (int o = 1; o < PSL_WAVE; o <<= 1) x += __shfl_xor(x, o, PSL_WAVE);
    if (lane_id() == 0) red[w][j] = x;
  }
  __syncthreads();
  if (threadIdx.x < SEL_COUNTS && tile < T) {
    int x = 0;
#pragma unroll
    for (int v = 0; v < PSL_BLOCK / PSL_WAVE; ++v) x += red[v][threadIdx.x];
    a.cnt[(int64_t)threadIdx.x * T + tile] = x;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[(int64_t)SEL_COUNTS * T] = 0;
}

// out: bin lists; cout: chunk list; sel: offsets [0..NBINS], rows, nonzeros,
// chunks. Kept rows are swept now: their marks are cleared.
__global__ void __launch_bounds__(PSL_BLOCK) k_sel_scatter(Dev d, SelArgs a, int T, BinEnt* out, LongChunk* cout,
                                                           int32_t* sel) {
  __shared__ int wc[SEL_ITEMS][NBINS + 1][PSL_BLOCK / PSL_WAVE];  // per item row, bin (and chunks), wave
  const int32_t* off = a.cnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int64_t R = (int64_t)NBINS * T, C = (int64_t)(NBINS + 1) * T, Z = (int64_t)(NBINS + 2) * T;
    for (int b = 0; b < NBINS; ++b) sel[b] = off[(int64_t)b * T];
    sel[NBINS] = off[R];
    sel[NBINS + 1] = off[R];
    sel[NBINS + 2] = off[Z] - off[C];
    sel[NBINS + 3] = off[C] - off[R];
  }
  int tile = blockIdx.x;
  if (tile >= T) return;
  __shared__ int marked;
  if (threadIdx.x == 0) {
    marked = d.dirty_tile[tile];
    d.dirty_tile[tile] = 0;  // the tile's marks are taken now (rows not kept keep
                             // theirs, harmlessly: a change marks them again)
  }
  __syncthreads();
  if ((sel_mode(a) & 1) && !marked) return;
  int w = threadIdx.x >> 6;
  int kb[SEL_ITEMS], nch[SEL_ITEMS], pre[SEL_ITEMS], cpre[SEL_ITEMS], r0[SEL_ITEMS], r1[SEL_ITEMS];
  int64_t row[SEL_ITEMS];
  bool any = false;
#pragma unroll
  for (int k = 0; k < SEL_ITEMS; ++k) {
    row[k] = (int64_t)tile * SEL_TILE + k * PSL_BLOCK + threadIdx.x;
    kb[k] = a.keep[row[k]];
    any |= kb[k] != 0;
  }
  if (!__syncthreads_or(any)) return;  // nothing kept in this tile
#pragma unroll
  for (int k = 0; k < SEL_ITEMS; ++k) {
    int64_t jj = kb[k] ? row[k] : 0;  // a row not kept reads row 0 (cached)
    r0[k] = d.rp[jj];
    r1[k] = d.rp[jj + 1];
  }
#pragma unroll
  for (int k = 0; k < SEL_ITEMS; ++k) {
    nch[k] = 0;
    if (kb[k] == 1 + BIN_LONG) nch[k] = d.lrow[long_row_index(d, (int)row[k])].nchunk;
    // rank among this wave's lanes of the same bin, and the chunk counts
    // before this lane in the wave (inclusive scan minus own)
    int b = kb[k] - 1;
    pre[k] = 0;
#pragma unroll
    for (int bb = 0; bb < NBINS; ++bb) {
      unsigned long long bal = __ballot(b == bb);
      if (b == bb) pre[k] = __popcll(bal & lanemask_lt());
      if (lane_id() == 0) wc[k][bb][w] = __popcll(bal);
    }
    int x = nch[k];
#pragma unroll
    for (int o = 1; o < PSL_WAVE; o <<= 1) {
      int y = __shfl_up(x, o, PSL_WAVE);
      if (lane_id() >= o) x += y;
    }
    cpre[k] = x - nch[k];
    if (lane_id() == PSL_WAVE - 1) wc[k][NBINS][w] = x;
  }
  __syncthreads();
  // exclusive prefix of every (item row, wave) count in row order, per bin
  // (and for the chunks): one thread per bin
  if (threadIdx.x <= NBINS) {
    int run = 0;
#pragma unroll
    for (int kk = 0; kk < SEL_ITEMS; ++kk)
#pragma unroll
      for (int v = 0; v < PSL_BLOCK / PSL_WAVE; ++v) {
        int x = wc[kk][threadIdx.x][v];
        wc[kk][threadIdx.x][v] = run;
        run += x;
      }
  }
  __syncthreads();
  int cbase = off[(int64_t)NBINS * T + tile] - off[(int64_t)NBINS * T];
#pragma unroll
  for (int k = 0; k < SEL_ITEMS; ++k) {
    int b = kb[k] - 1;
    if (b < 0) continue;
    int64_t i = row[k];
    int start = r0[k];
    int len = r1[k] - start;
    out[off[(int64_t)b * T + tile] + wc[k][b][w] + pre[k]] = BinEnt{(int)i, start, len, 0};
    d.dirty[i] = 0;
    if (nch[k]) {
      LongRow lr = d.lrow[long_row_index(d, (int)i)];
      int cb = wc[k][NBINS][w] + cpre[k];
      for (int c = 0; c < lr.nchunk; ++c) cout[cbase + cb + c] = d.chunks0[lr.chunk0 + c];
    }
  }
}

void select_rows(const Dev& d, const int32_t* mode_dev, int mode_host, int t_long, int t_g8, uint8_t* keep,
                 int32_t* cnt, BinEnt* out, LongChunk* cout, int32_t* sel, int32_t* ws, hipStream_t s) {
  SelArgs a{mode_dev, mode_host, t_long, t_g8, keep, cnt};
  int T = (int)((d.m + SEL_TILE - 1) / SEL_TILE);
  unsigned grid = (unsigned)(T > 0 ? T : 1);
  hipLaunchKernelGGL(k_sel_count, dim3(grid), dim3(PSL_BLOCK), 0, s, d, a, T);
  scan_excl(cnt, cnt, (int64_t)SEL_COUNTS * T + 1, nullptr, ws, s);
  hipLaunchKernelGGL(k_sel_scatter, dim3(grid), dim3(PSL_BLOCK), 0, s, d, a, T, out, cout, sel);
}

// Rows of the columns whose bounds changed (or that were fixed) this round,
// from the transposed copy; their infinite-contribution counts follow the
// bounds that became finite. One wavefront per 64 columns walks the entries of
// its changed columns; columns of more than MARK_DENSE entries (listed once
// at ingest) are walked by every workgroup of a second launch.
#define MARK_DENSE 4096
#define MARK_SHORT 16
#define MARK_MASK (CC_LB | CC_UB | CC_FIX)

// One entry (q, row i) of a changed column: mark the row (when the next
// round sweeps dirty rows only), and (with count) lower its infinite-
// contribution counts when the column's lb / ub became finite.
__device__ __forceinline__ void mark_entry(const Dev& d, int64_t q, int code, bool mark, bool count) {
  int i = d.ri[q];
  if (mark) {
    d.dirty[i] = 1;
    d.dirty_tile[i >> 10] = 1;
  }
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

// exclusive prefix (lanes below) and total of per-lane values 0..31 across
// the wavefront, from one ballot per bit
__device__ __forceinline__ void wave_scan5(int v, int& pre, int& tot) {
  unsigned long long below = lanemask_lt();
  pre = tot = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    unsigned long long m = __ballot((v >> b) & 1);
    pre += __popcll(m & below) << b;
    tot += __popcll(m) << b;
  }
}

// A lane reads the codes of MARK_COLS consecutive columns as one word (the
// code array is 256-byte aligned and padded, so a word starting below n stays
// inside it); the wavefront's columns to walk are listed in LDS and taken 64
// at a time, one per lane.
#define MARK_COLS 4
#define MARK_TILE (PSL_BLOCK * MARK_COLS)

__global__ void __launch_bounds__(PSL_BLOCK) k_mark_sparse(Dev d, RoundMode rm) {
  int mode = round_mode(d, rm);
  if (blockIdx.x == 0 && threadIdx.x == 0) d.flags->mode = mode;
  if (mode == 0) return;
  __shared__ int32_t list[MARK_TILE];
  int lane = lane_id();
  int32_t* wl = list + (threadIdx.x >> 6) * (PSL_WAVE * MARK_COLS);
  int64_t j0 = (int64_t)blockIdx.x * MARK_TILE + (int64_t)threadIdx.x * MARK_COLS;
  uint32_t cw = 0;
  if (j0 < d.n) {
    int64_t rem = d.n - j0;
    cw = reinterpret_cast<const uint32_t*>(d.col_code)[j0 >> 2];
    if (rem < 4) cw &= (1u << (8 * (int)rem)) - 1u;
  }
  int nm = 0;
#pragma unroll
  for (int b = 0; b < MARK_COLS; ++b) nm += mark_col((cw >> (8 * b)) & 0xFF, mode);
  int mpre, mtot;
  wave_scan5(nm, mpre, mtot);
#pragma unroll
  for (int b = 0; b < MARK_COLS; ++b)
    if (mark_col((cw >> (8 * b)) & 0xFF, mode)) wl[mpre++] = (int32_t)(j0 + b);
  __syncthreads();
  for (int c0 = 0; c0 < mtot; c0 += PSL_WAVE) {
    int q0 = 0, q1 = 0, code = 0;
    if (c0 + lane < mtot) {
      int j = wl[c0 + lane];
      code = d.col_code[j];
      q0 = d.cp[j];
      q1 = d.cp[j + 1];
    }
    int len = q1 - q0;
    // short columns: the entries of the lanes' columns, concatenated in
    // column order, one per lane (a column's entries are contiguous, so the
    // row-index loads of a step touch a few lines, and no lane walks a
    // column alone)
    int sl = len <= MARK_SHORT ? len : 0;
    int pre, tot;
    wave_scan5(sl, pre, tot);
    for (int e0 = 0; e0 < tot; e0 += PSL_WAVE) {
      int e = e0 + lane;
      // the entry's column: the last lane whose prefix is <= e
      int lo = 0, hi = PSL_WAVE - 1;
#pragma unroll
      for (int it = 0; it < 6; ++it) {
        int mid = (lo + hi + 1) >> 1;
        bool le = __shfl(pre, mid, PSL_WAVE) <= e;
        lo = le ? mid : lo;
        hi = le ? hi : mid - 1;
      }
      int q = __shfl(q0, lo, PSL_WAVE) + (e - __shfl(pre, lo, PSL_WAVE));
      int cl = __shfl(code, lo, PSL_WAVE);
      if (e < tot) mark_entry(d, q, cl, mode & 1, mode & 2);
    }
    // longer ones: the wavefront walks them one after another
    unsigned long long mask = __ballot(len > MARK_SHORT && len <= MARK_DENSE);
    while (mask) {
      int l = __ffsll((long long)mask) - 1;
      mask &= mask - 1;
      int a = __shfl(q0, l, PSL_WAVE), b = __shfl(q1, l, PSL_WAVE), cl = __shfl(code, l, PSL_WAVE);
      for (int q = a + lane; q < b; q += PSL_WAVE) mark_entry(d, q, cl, mode & 1, mode & 2);
    }
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

void mark_dirty(const Dev& d, bool allow_incremental, int incr_factor, int count_factor, hipStream_t s) {
  RoundMode rm{allow_incremental ? 1 : 0, incr_factor, count_factor};
  unsigned blocks = (unsigned)((d.n + MARK_TILE - 1) / MARK_TILE);
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
    d.dirty[t] = 0;
    d.fs_pick[t] = 0x7FFFFFFF;
  }
  if (t <= d.m / 1024) d.dirty_tile[t] = 0;
  if (t < d.n) {
    double2 b = d.bnd[t];
    d.touch[t] = 1;    // the first round decides every column
    d.fs_flag[t] = 1;  // and checks every column for a free singleton
    d.owner[t] = ~0ull;
    d.lsrc[t] = is_inf(b.x) ? -1 : -2;
    d.usrc[t] = is_inf(b.y) ? -1 : -2;
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
    f.fin_cols = f.mode = f.lead_count = f.fs_total = f.fs_rows = f.fs_claims = 0;
    f.error_pos = 0x7FFFFFFFFFFFFFFFLL;
    *d.flags = f;
  }
}

// Variable locks of every column from the alive rows (dual fixing): one bit
// per position of the transposed copy for each direction, scanned, and each
// column's count read off as the difference of the scans at its ends.
__global__ void k_lock_bits(Dev d, int32_t* dn, int32_t* up) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= d.nnz; q += stride) {
    unsigned long long b = 0;
    if (q < d.nnz) {
      int i = d.ri[q];
      if (d.row_on[i]) b = lock_bits(d.cva[q], d.lhs[i], d.rhs[i]);
    }
    dn[q] = (int32_t)(b & 1ull);
    up[q] = (int32_t)(b >> 32);
  }
}

__global__ void k_lock_cols(Dev d, const int32_t* dn, const int32_t* up) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  int q0 = d.cp[j], q1 = d.cp[j + 1];
  unsigned long long down = (unsigned)(dn[q1] - dn[q0]), upc = (unsigned)(up[q1] - up[q0]);
  d.locks[j] = down | (upc << 32);
}

void init_locks(const Dev& d, int32_t* dn, int32_t* up, int32_t* ws, hipStream_t s) {
  if (d.n == 0) return;
  int64_t blocks = (d.nnz + 1 + PSL_BLOCK - 1) / PSL_BLOCK;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_lock_bits, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, d, dn, up);
  scan_excl(dn, dn, d.nnz + 1, nullptr, ws, s);
  scan_excl(up, up, d.nnz + 1, nullptr, ws, s);
  hipLaunchKernelGGL(k_lock_cols, dim3((unsigned)((d.n + PSL_BLOCK - 1) / PSL_BLOCK)), dim3(PSL_BLOCK), 0, s, d,
                     (const int32_t*)dn, (const int32_t*)up);
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
