// primitives.hip -- device-wide scan, stable radix pass, fill and canonical
// pairwise array sum. Plain reduce-then-scan; every result is independent of
// scheduling (integer sums, and pairwise trees over aligned power-of-two
// blocks).
#include "psl_kern.h"

namespace psl {

#define SCAN_ITEMS 8
#define SCAN_TILE (PSL_BLOCK * SCAN_ITEMS)

static_assert(SCAN_ITEMS == 8, "load8 / store8 move eight ints");

// eight consecutive ints from base (zero beyond n): two 16-byte loads when
// all eight are in range and aligned, else one at a time
__device__ __forceinline__ void load8(const int32_t* in, int64_t base, int64_t n, int (&v)[SCAN_ITEMS]) {
  if (base + SCAN_ITEMS <= n && (((uintptr_t)(in + base)) & 15) == 0) {
    int4 a = *(const int4*)(in + base);
    int4 b = *(const int4*)(in + base + 4);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
    v[4] = b.x;
    v[5] = b.y;
    v[6] = b.z;
    v[7] = b.w;
    return;
  }
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = base + k < n ? in[base + k] : 0;
}

__device__ __forceinline__ void store8(int32_t* out, int64_t base, int64_t n, const int (&v)[SCAN_ITEMS]) {
  if (base + SCAN_ITEMS <= n && (((uintptr_t)(out + base)) & 15) == 0) {
    *(int4*)(out + base) = make_int4(v[0], v[1], v[2], v[3]);
    *(int4*)(out + base + 4) = make_int4(v[4], v[5], v[6], v[7]);
    return;
  }
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) out[base + k] = v[k];
}

__global__ void __launch_bounds__(PSL_BLOCK) k_scan_tile_sums(const int32_t* in, int64_t n, int32_t* sums) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load8(in, base, n, v);
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
  int tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(PSL_BLOCK) k_scan_tile_apply(const int32_t* in, int32_t* out, int64_t n,
                                                               const int32_t* tile_off, int32_t* total) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load8(in, base, n, v);
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
  int tot;
  int pre = block_excl_scan(s, &tot);
  int off = tile_off ? tile_off[blockIdx.x] : 0;
  int run = off + pre;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int x = v[k];
    v[k] = run;
    run += x;
  }
  store8(out, base, n, v);
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

__global__ void k_fill_i32(int32_t* out, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = v;
}

size_t scan_ws_ints(int64_t n) {
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb <= 1) return 0;
  return (size_t)nb + scan_ws_ints(nb);
}

void fill_i32(int32_t* out, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + PSL_BLOCK - 1) / PSL_BLOCK;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(PSL_BLOCK), 0, s, out, v, n);
}

// Up to SCAN_ONE_MAX ints: one workgroup stages the array in LDS with
// coalesced loads, each thread scans a contiguous run of it, and one block
// scan joins the runs (one launch and one trip to memory instead of three
// launches).
#define SCAN_ONE_MAX 12288

__global__ void __launch_bounds__(PSL_BLOCK) k_scan_one(const int32_t* in, int32_t* out, int64_t n, int32_t* total) {
  __shared__ int32_t buf[SCAN_ONE_MAX];
  int nn = (int)n;
  {
    // every load in flight at once
    int v[SCAN_ONE_MAX / PSL_BLOCK];
#pragma unroll
    for (int i = 0; i < SCAN_ONE_MAX / PSL_BLOCK; ++i) {
      int k = i * PSL_BLOCK + threadIdx.x;
      v[i] = k < nn ? in[k] : 0;
    }
#pragma unroll
    for (int i = 0; i < SCAN_ONE_MAX / PSL_BLOCK; ++i) {
      int k = i * PSL_BLOCK + threadIdx.x;
      if (k < nn) buf[k] = v[i];
    }
  }
  __syncthreads();
  int per = (nn + PSL_BLOCK - 1) / PSL_BLOCK;
  int b0 = threadIdx.x * per;
  int b1 = b0 + per < nn ? b0 + per : nn;
  int s = 0;
  for (int k = b0; k < b1; ++k) s += buf[k];
  int tot;
  int run = block_excl_scan(s, &tot);
  for (int k = b0; k < b1; ++k) {
    int v = buf[k];
    buf[k] = run;
    run += v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nn; k += PSL_BLOCK) out[k] = buf[k];
  if (total && threadIdx.x == 0) *total = tot;
}

void scan_excl(const int32_t* in, int32_t* out, int64_t n, int32_t* total, int32_t* ws, hipStream_t s) {
  if (n <= 0) {
    if (total) fill_i32(total, 0, 1, s);
    return;
  }
  if (n <= SCAN_ONE_MAX) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(PSL_BLOCK), 0, s, in, out, n, total);
    return;
  }
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  int32_t* sums = ws;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)nb), dim3(PSL_BLOCK), 0, s, in, n, sums);
  scan_excl(sums, sums, nb, nullptr, ws + nb, s);
  hipLaunchKernelGGL(k_scan_tile_apply, dim3((unsigned)nb), dim3(PSL_BLOCK), 0, s, in, out, n,
                     (const int32_t*)sums, total);
}

// ---------------------------------------------------------------------------
// stable radix pass
// ---------------------------------------------------------------------------

#define RX_ROUNDS 8
#define RX_TILE (PSL_BLOCK * RX_ROUNDS)

__global__ void __launch_bounds__(PSL_BLOCK) k_rx_count(const uint32_t* keys, int64_t n, int shift, uint32_t mask,
                                                        int32_t* hist, int ntiles) {
  __shared__ int c[256];
  int t = threadIdx.x;
  c[t] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RX_TILE;
  for (int r = 0; r < RX_ROUNDS; ++r) {
    int64_t idx = base + r * PSL_BLOCK + t;
    if (idx < n) atomicAdd(&c[(keys[idx] >> shift) & mask], 1);
  }
  __syncthreads();
  if ((uint32_t)t <= mask) hist[(int64_t)t * ntiles + blockIdx.x] = c[t];
}

__global__ void __launch_bounds__(PSL_BLOCK) k_rx_scatter(const uint32_t* kin, const int32_t* vin, uint32_t* kout,
                                                          int32_t* vout, int64_t n, int shift, uint32_t mask,
                                                          const int32_t* hoff, int ntiles) {
  __shared__ int tile_cnt[256];
  __shared__ int wcnt[PSL_BLOCK / PSL_WAVE][256];
  int t = threadIdx.x, w = t >> 6;
  tile_cnt[t] = 0;
#pragma unroll
  for (int k = 0; k < PSL_BLOCK / PSL_WAVE; ++k) wcnt[k][t] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RX_TILE;
  for (int r = 0; r < RX_ROUNDS; ++r) {
    int64_t idx = base + r * PSL_BLOCK + t;
    bool valid = idx < n;
    uint32_t key = valid ? kin[idx] : 0u;
    int32_t val = valid ? (vin ? vin[idx] : (int32_t)idx) : 0;
    uint32_t d = (key >> shift) & mask;
    // lanes of this wave holding the same digit
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1u;
      unsigned long long bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    int rank = __popcll(peers & lanemask_lt());
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    int pos = 0;
    if (valid) {
      int before = tile_cnt[d];
      for (int k = 0; k < w; ++k) before += wcnt[k][d];
      pos = hoff[(int64_t)d * ntiles + blockIdx.x] + before + rank;
    }
    __syncthreads();
    {
      int sum = 0;
#pragma unroll
      for (int k = 0; k < PSL_BLOCK / PSL_WAVE; ++k) {
        sum += wcnt[k][t];
        wcnt[k][t] = 0;
      }
      tile_cnt[t] += sum;
    }
    __syncthreads();
    if (valid) {
      kout[pos] = key;
      vout[pos] = val;
    }
  }
}

size_t radix_ws_ints(int64_t n) {
  int64_t ntiles = (n + RX_TILE - 1) / RX_TILE;
  if (ntiles < 1) ntiles = 1;
  return (size_t)(256 * ntiles) + scan_ws_ints(256 * ntiles);
}

void radix_pass(const uint32_t* keys_in, const int32_t* vals_in, uint32_t* keys_out, int32_t* vals_out,
                int64_t n, int shift, int bits, int32_t* ws, hipStream_t s) {
  if (n <= 0) return;
  int ntiles = (int)((n + RX_TILE - 1) / RX_TILE);
  uint32_t mask = (1u << bits) - 1u;
  int32_t* hist = ws;
  int32_t* sws = ws + 256 * (int64_t)ntiles;
  hipLaunchKernelGGL(k_rx_count, dim3(ntiles), dim3(PSL_BLOCK), 0, s, keys_in, n, shift, mask, hist, ntiles);
  scan_excl(hist, hist, (int64_t)(mask + 1) * ntiles, nullptr, sws, s);
  hipLaunchKernelGGL(k_rx_scatter, dim3(ntiles), dim3(PSL_BLOCK), 0, s, keys_in, vals_in, keys_out, vals_out, n,
                     shift, mask, (const int32_t*)hist, ntiles);
}

// Stable pass with a (row, value) payload, staged through LDS: each tile is
// ordered by digit in LDS first, so consecutive threads store consecutive
// positions of a digit's run (coalesced) instead of one scattered store per
// item. With rows_in == nullptr the payload of item p is (rowid1[p + 1],
// vals_in[p]) (the CSR itself).
__global__ void __launch_bounds__(PSL_BLOCK) k_tx_scatter(const uint32_t* kin, const int32_t* rin,
                                                          const int32_t* rowid1, const double* vin, uint32_t* kout,
                                                          int32_t* rout, double* vout, int64_t n, int shift,
                                                          uint32_t mask, const int32_t* hoff, int ntiles) {
  __shared__ int start[256];   // tile-local start of each digit's run
  __shared__ int gbase[256];   // global start of the tile's run of each digit
  __shared__ int run[256];     // items of each digit placed so far
  __shared__ int wcnt[PSL_BLOCK / PSL_WAVE][256];
  __shared__ uint32_t sk[RX_TILE];
  __shared__ int32_t sr[RX_TILE];
  __shared__ double sv[RX_TILE];
  int t = threadIdx.x, w = t >> 6;
  int64_t base = (int64_t)blockIdx.x * RX_TILE;
  int cnt = (int)(n - base < RX_TILE ? n - base : RX_TILE);
  uint32_t key[RX_ROUNDS];
#pragma unroll
  for (int r = 0; r < RX_ROUNDS; ++r) {
    int64_t idx = base + r * PSL_BLOCK + t;
    key[r] = idx < n ? kin[idx] : 0u;
  }
  start[t] = 0;
  run[t] = 0;
  gbase[t] = (uint32_t)t <= mask ? hoff[(int64_t)t * ntiles + blockIdx.x] : 0;
#pragma unroll
  for (int k = 0; k < PSL_BLOCK / PSL_WAVE; ++k) wcnt[k][t] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RX_ROUNDS; ++r)
    if (r * PSL_BLOCK + t < cnt) atomicAdd(&start[(key[r] >> shift) & mask], 1);
  __syncthreads();
  {
    int h = start[t], tot;
    int e = block_excl_scan(h, &tot);
    start[t] = e;
  }
  __syncthreads();
  int slot[RX_ROUNDS];
#pragma unroll
  for (int r = 0; r < RX_ROUNDS; ++r) {
    bool valid = r * PSL_BLOCK + t < cnt;
    uint32_t d = (key[r] >> shift) & mask;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1u;
      unsigned long long bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    int rank = __popcll(peers & lanemask_lt());
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    slot[r] = -1;
    if (valid) {
      int before = start[d] + run[d];
      for (int k = 0; k < w; ++k) before += wcnt[k][d];
      slot[r] = before + rank;
    }
    __syncthreads();
    {
      int sum = 0;
#pragma unroll
      for (int k = 0; k < PSL_BLOCK / PSL_WAVE; ++k) {
        sum += wcnt[k][t];
        wcnt[k][t] = 0;
      }
      run[t] += sum;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RX_ROUNDS; ++r) {
    if (slot[r] < 0) continue;
    int64_t idx = base + r * PSL_BLOCK + t;
    sk[slot[r]] = key[r];
    sr[slot[r]] = rin ? rin[idx] : rowid1[idx + 1];
    sv[slot[r]] = vin[idx];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RX_ROUNDS; ++r) {
    int sl = r * PSL_BLOCK + t;
    if (sl >= cnt) continue;
    uint32_t k = sk[sl];
    uint32_t d = (k >> shift) & mask;
    int64_t g = (int64_t)gbase[d] + (sl - start[d]);
    kout[g] = k;
    rout[g] = sr[sl];
    vout[g] = sv[sl];
  }
}

void radix_pass_payload(const uint32_t* keys_in, const int32_t* rows_in, const int32_t* rowid1,
                        const double* vals_in, uint32_t* keys_out, int32_t* rows_out, double* vals_out, int64_t n,
                        int shift, int bits, int32_t* ws, hipStream_t s) {
  if (n <= 0) return;
  int ntiles = (int)((n + RX_TILE - 1) / RX_TILE);
  uint32_t mask = (1u << bits) - 1u;
  int32_t* hist = ws;
  int32_t* sws = ws + 256 * (int64_t)ntiles;
  hipLaunchKernelGGL(k_rx_count, dim3(ntiles), dim3(PSL_BLOCK), 0, s, keys_in, n, shift, mask, hist, ntiles);
  scan_excl(hist, hist, (int64_t)(mask + 1) * ntiles, nullptr, sws, s);
  hipLaunchKernelGGL(k_tx_scatter, dim3(ntiles), dim3(PSL_BLOCK), 0, s, keys_in, rows_in, rowid1, vals_in, keys_out,
                     rows_out, vals_out, n, shift, mask, (const int32_t*)hist, ntiles);
}

// ---------------------------------------------------------------------------
// canonical pairwise sum of an array
// ---------------------------------------------------------------------------

#define PW_TILE 2048

// Sum of one aligned tile x[0..2048) (elements at or beyond lim read as 0) by
// the whole block: eight contiguous leaves per thread (tree of 8), a butterfly
// over the wave (tree of 64 such groups), then the four wave sums as
// (w0 + w1) + (w2 + w3). Every thread returns the sum.
__device__ __forceinline__ double tile_sum(const double* x, int64_t lim) {
  __shared__ double ws[PSL_BLOCK / PSL_WAVE];
  int64_t base = (int64_t)threadIdx.x * 8;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = base + k < lim ? x[base + k] : 0.0;
  double s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  s = group_sum<PSL_WAVE>(s);
  if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = (ws[0] + ws[1]) + (ws[2] + ws[3]);
  __syncthreads();
  return t;
}

// Each block sums the aligned chunk [2048 b, 2048 b + 2048).
__global__ void __launch_bounds__(PSL_BLOCK) k_pw_chunks(const double* x, int64_t n, double* out) {
  int64_t base = (int64_t)blockIdx.x * PW_TILE;
  double t = tile_sum(x + base, n - base);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

size_t pairwise_ws_doubles(int64_t n) {
  int64_t nb = (n + PW_TILE - 1) / PW_TILE;
  if (nb <= 1) return 1;
  return (size_t)nb + pairwise_ws_doubles(nb);
}

void pairwise_sum(const double* x, int64_t n, double* out, double* ws, hipStream_t s) {
  int64_t nb = (n + PW_TILE - 1) / PW_TILE;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_pw_chunks, dim3(1), dim3(PSL_BLOCK), 0, s, x, n, out);
    return;
  }
  hipLaunchKernelGGL(k_pw_chunks, dim3((unsigned)nb), dim3(PSL_BLOCK), 0, s, x, n, ws);
  pairwise_sum(ws, nb, out, ws + nb, s);
}

// One block per segment of at most 2048 tiles: the tile sums go to LDS, then
// one more tile tree over them (the same tree as pairwise_sum's second level).
__global__ void __launch_bounds__(PSL_BLOCK) k_pw_segments(const double* x, const int32_t* seg, const double* off,
                                                           double* out) {
  __shared__ double tiles[PW_TILE];
  int k = blockIdx.x;
  int64_t s0 = seg[k], n = (int64_t)seg[k + 1] - s0;
  int64_t nt = (n + PW_TILE - 1) / PW_TILE;
  if (nt > PW_TILE) return;  // summed on its own
  for (int64_t t = 0; t < nt; ++t) {
    double v = tile_sum(x + s0 + t * PW_TILE, n - t * PW_TILE);
    if (threadIdx.x == 0) tiles[t] = v;
  }
  __syncthreads();
  double sum = nt <= 1 ? (nt == 1 ? tiles[0] : 0.0) : tile_sum(tiles, nt);
  if (threadIdx.x == 0) out[k] = pos0(off[k] + sum);
}

__global__ void k_pw_finish(const double* sum, const double* off, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = pos0(off[0] + sum[0]);
}

void segmented_pairwise_sum(const double* x, const int32_t* seg_dev, const int32_t* seg_host, int K,
                            const double* off, double* out, double* ws, hipStream_t s) {
  if (K <= 0) return;
  hipLaunchKernelGGL(k_pw_segments, dim3((unsigned)K), dim3(PSL_BLOCK), 0, s, x, seg_dev, off, out);
  for (int k = 0; k < K; ++k) {
    int64_t n = (int64_t)seg_host[k + 1] - seg_host[k];
    if ((n + PW_TILE - 1) / PW_TILE <= PW_TILE) continue;
    pairwise_sum(x + seg_host[k], n, ws, ws + 1, s);
    hipLaunchKernelGGL(k_pw_finish, dim3(1), dim3(64), 0, s, (const double*)ws, off + k, out + k);
  }
}

}  // namespace psl
