// capi.hip -- libpsl's C-ABI: device arena, ingest, the round controller
// (section 3.1: rounds until nothing tightens or a cap is hit; then parallel
// rows, section 3.2; repeated for a few outer cycles), compaction and the
// host postsolve (section 3.3).
//
// Control crosses to the host once per round: a 64-byte flag block (records
// emitted, infeasible / unbounded) is read back to decide whether to go on.
//
// One engine serves a single LP (K = 1) and batches of K LPs laid out as the
// blocks of one block-diagonal LP. In a batch every LP has its own state
// machine on the host (propagating / converged / done, its round count and
// outer cycles); the per-round readback then also holds each LP's record
// count and flags, and LPs that stopped are filtered out of the bin lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "engine.h"

using namespace psl;

namespace {

thread_local std::string g_create_error = "no error";

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

#define HIPCHK(p, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      (p)->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call; \
      return PSL_ERR_DEVICE;                                                         \
    }                                                                                \
  } while (0)

static psl_status fail(psl_presolver* p, psl_status st, const std::string& msg) {
  p->err = msg;
  return st;
}

template <class T>
static psl_status dalloc(psl_presolver* p, T** out, size_t count) {
  void* ptr = nullptr;
  size_t bytes = count * sizeof(T);
  if (bytes == 0) bytes = 64;
  bytes = (bytes + 255) & ~(size_t)255;
  if (p->carve) {  // static-scratch mode: the next 256-byte aligned piece
    if (bytes > p->carve_cap - p->carve_used) {
      p->err = "the static scratch (" + std::to_string(p->carve_cap) + " bytes) is too small for this LP";
      return PSL_ERR_CAPACITY;
    }
    *out = (T*)(p->carve + p->carve_used);
    p->carve_used += bytes;
    p->arena_bytes += bytes;
    return PSL_OK;
  }
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
    return PSL_ERR_OOM;
  }
  p->allocs.push_back(ptr);
  p->arena_bytes += bytes;
  *out = (T*)ptr;
  return PSL_OK;
}

#define ALLOC(ptr, cnt)                               \
  do {                                                \
    psl_status st_ = dalloc(p, &(ptr), (size_t)(cnt)); \
    if (st_ != PSL_OK) return st_;                    \
  } while (0)

extern "C" void psl_settings_default(psl_settings* s) {
  if (!s) return;
  std::memset(s, 0, sizeof *s);
  s->max_rounds = 16;
  s->max_outer = 4;
  s->enable_parallel_rows = 1;
  s->feas_tol = 1e-9;
  s->fix_tol = 1e-9;
  s->min_improve = 1e-7;
  s->par_tol = 1e-9;
  s->inf_value = 1e20;
  s->coef_tol = 1e-9;
  s->bin_thresholds = nullptr;
  s->n_bins = 0;
  s->device = 0;
  s->stream = nullptr;
  s->split_sweep = 0;
  s->enable_dual_fix = 0;
  s->enable_free_singletons = 0;
  s->enable_parallel_cols = 0;
  s->enable_forcing_rows = 0;
  s->enable_doubletons = 0;
  s->device_records = 0;
  s->enable_dominated = 0;
}

std::string psl::check_settings(const psl_settings* s) {
  if (s->max_rounds < 1 || s->max_outer < 1 || (int64_t)s->max_outer * (s->max_rounds + 1) + 1 > 65535)
    return "invalid round limits";
  if (!(s->feas_tol >= 0) || !(s->fix_tol >= 0) || !(s->min_improve >= 0) || !(s->par_tol >= 0) ||
      !(s->inf_value > 0) || !(s->coef_tol >= 0))
    return "invalid tolerance";
  if (s->enable_dual_fix != 0 && s->enable_dual_fix != 1) return "enable_dual_fix must be 0 or 1";
  if (s->enable_free_singletons != 0 && s->enable_free_singletons != 1)
    return "enable_free_singletons must be 0 or 1";
  if (s->enable_parallel_cols != 0 && s->enable_parallel_cols != 1) return "enable_parallel_cols must be 0 or 1";
  if (s->enable_forcing_rows != 0 && s->enable_forcing_rows != 1) return "enable_forcing_rows must be 0 or 1";
  if (s->enable_doubletons != 0 && s->enable_doubletons != 1) return "enable_doubletons must be 0 or 1";
  if (s->device_records < 0) return "device_records must be >= 0";
  if (s->enable_dominated != 0 && s->enable_dominated != 1) return "enable_dominated must be 0 or 1";
  if (s->bin_thresholds) {
    if (s->n_bins != 2 && s->n_bins != 3) return "bin_thresholds needs n_bins = 2 or 3";
    int a = s->bin_thresholds[0], b = s->bin_thresholds[1];
    if (s->n_bins == 3 && s->bin_thresholds[2] != 4 && s->bin_thresholds[2] != 8)
      return "bin_thresholds[2] (longest row of the 8-lane bin) must be 4 (no such bin) or 8";
    if (a < 16 || a > 512) return "bin_thresholds[0] (longest wavefront row) must be in [16, 512]";
    if (b < PASS_LEN || b > PASS_LEN * long_max_passes() || (b & (b - 1)) != 0)
      return "bin_thresholds[1] (chunk positions) must be a power of two >= 2048";
  }
  return "";
}

std::string psl::check_lp_shape(const psl_lp* lp) {
  if (lp->m < 0 || lp->n < 0 || lp->nnz < 0) return "negative size";
  if (lp->nnz >= ((int64_t)1 << 30)) return "nnz must be below 2^30";
  if (lp->m >= (1 << 30) || lp->n >= (1 << 30)) return "m and n must be below 2^30";
  if (lp->m == 0 && lp->nnz != 0) return "entries without rows";
  if (lp->m > 0 && (!lp->row_ptr || !lp->lhs || !lp->rhs)) return "null row array";
  if (lp->n > 0 && (!lp->lb || !lp->ub || !lp->c)) return "null column array";
  if (lp->nnz > 0 && (!lp->col_idx || !lp->val)) return "null matrix array";
  if (lp->mem != PSL_MEM_HOST && lp->mem != PSL_MEM_DEVICE) return "bad mem kind";
  if (!std::isfinite(lp->obj_offset)) return "offset not finite";
  return "";
}

template <class T>
static psl_status halloc(psl_presolver* p, T** out, size_t count) {
  size_t bytes = count * sizeof(T);
  if (bytes == 0) bytes = 64;
  if (p->hcarve) {  // static-scratch mode: host staging from a static buffer
    bytes = (bytes + 63) & ~(size_t)63;
    if (bytes > p->hcarve_cap - p->hcarve_used) {
      p->err = "internal: static host staging too small";
      return PSL_ERR_CAPACITY;
    }
    *out = (T*)(p->hcarve + p->hcarve_used);
    p->hcarve_used += bytes;
    return PSL_OK;
  }
  if (hipHostMalloc((void**)out, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    p->err = "pinned host allocation failed";
    return PSL_ERR_OOM;
  }
  p->hallocs.push_back((void*)*out);
  return PSL_OK;
}

#define HALLOC(ptr, cnt)                               \
  do {                                                 \
    psl_status st_ = halloc(p, &(ptr), (size_t)(cnt)); \
    if (st_ != PSL_OK) return st_;                     \
  } while (0)

// device arena for LPs of up to cap_m rows, cap_n columns, cap_nnz entries
// (and cap_K LPs)
static psl_status setup_arena(psl_presolver* p) {
  int64_t m = p->cap_m, n = p->cap_n, N = p->cap_nnz, K = p->cap_K;
  Dev& d = p->d;
  int32_t *rp, *ci, *cp, *ri, *col_len, *src, *cnt, *off;
  double *va, *cva, *lhs, *rhs;
  double2* bnd;
  long long* bkey;
  uint8_t *row_on, *row_code, *col_code;
  RowOut* row_out;
  Cand* cand;
  Flags* flags;
  ALLOC(rp, m + 1);
  ALLOC(ci, N);
  ALLOC(va, N);
  ALLOC(cp, n + 1);
  ALLOC(ri, N);
  ALLOC(cva, N);
  ALLOC(lhs, m);
  ALLOC(rhs, m);
  ALLOC(bnd, n);
  ALLOC(bkey, 2 * n);
  ALLOC(src, 2 * n);
  ALLOC(p->c_mut, n);
  ALLOC(p->c_work, n);
  ALLOC(col_len, n);
  ALLOC(row_on, m);
  ALLOC(row_code, m);
  ALLOC(col_code, n);
  ALLOC(row_out, m);
  // candidate regions: short and wavefront bins reserve at most 8 entries per
  // row plus 8 per position (their regions are sized for the bin's longest
  // row); long rows reserve 2 per position
  p->cand_cap = 8 * m + 10 * N + 8 * PASS_LEN;
  ALLOC(cand, p->cand_cap);
  // one count per sweep workgroup: at most m/4 + NBINS for the row bins plus
  // one per long-row chunk
  ALLOC(p->cand_cnt, m / 4 + NBINS + (N / PASS_LEN + N / 512 + 2) + 64);
  ALLOC(flags, 1);
  ALLOC(cnt, m + n + 1);
  ALLOC(off, m + n + 1);
  ALLOC(p->bins_a, m);
  ALLOC(p->bins_s, m);
  ALLOC(p->sel_dev, 16);
  ALLOC(p->sel_keep, select_keep_bytes(m));
  ALLOC(p->sel_cnt, select_count_ints(m));
  ALLOC(p->bin_counts_dev, NBINS);
  ALLOC(p->lb_in, n);
  ALLOC(p->ub_in, n);

  int64_t big = std::max<int64_t>(N, m) + 2;
  ALLOC(p->isc.rowid1, N + 2);
  ALLOC(p->isc.k0, big);
  ALLOC(p->isc.k1, big);
  ALLOC(p->isc.v0, big);
  ALLOC(p->isc.v1, big);
  size_t wsn = std::max<size_t>(scan_ws_ints(N + 1), radix_ws_ints(std::max<int64_t>(N, m)));
  wsn = std::max<size_t>(wsn, scan_ws_ints(m + n + 1));
  wsn = std::max<size_t>(wsn, par_cols_ws_ints(n)) + 64;
  ALLOC(p->ws, wsn);
  p->isc.ws = p->ws;

  // long rows are longer than the wavefront threshold; chunks of >= 2048
  p->long_cap = N / ((int64_t)p->thresholds[0] + 1) + 1;
  p->chunk_cap = N / PASS_LEN + p->long_cap + 1;
  ALLOC(p->chunks_a, p->chunk_cap);
  ALLOC(p->chunks_s, p->chunk_cap);
  ALLOC(p->chunks_0, p->chunk_cap);
  uint8_t* dirty;
  ALLOC(dirty, m);
  ALLOC(d.dirty_tile, m / 1024 + 2);
  ALLOC(d.touch, n);
  ALLOC(d.locks, n);
  ALLOC(d.lsrc, n);
  ALLOC(d.usrc, n);
  ALLOC(d.fs_flag, n);
  ALLOC(d.fs_pick, m);
  ALLOC(d.owner, n);
  ALLOC(d.fs_bad, m);
  ALLOC(d.rinf, m);
  ALLOC(d.dense_cols, N / 4096 + 2);
  ALLOC(d.n_dense, 1);
  LongPart* lpart;
  LongRow* lrow;
  ALLOC(lpart, p->chunk_cap);
  ALLOC(lrow, p->long_cap);


  // parallel rows: a table of >= 2m slots (per LP in a batch)
  int64_t cap = 64;
  while (cap < 2 * m) cap <<= 1;
  if (K > 1) cap = 4 * m + 64 * K + 64;
  p->par_slots = cap;
  ALLOC(p->par.table, cap);
  ALLOC(p->par.slot, m);
  ALLOC(p->par.lead, m);
  ALLOC(p->par.side_key, 2 * m);
  ALLOC(p->par.side_src, 2 * m);
  ALLOC(p->par.is_leader, m);
  ALLOC(p->par.vlist, m);
  ALLOC(p->par.hacc, 4 * p->long_cap);
  ALLOC(p->par.lam, m);
  ALLOC(p->par.abits, n / 64 + 1);
  p->par.lpt = nullptr;
  if (p->s.enable_doubletons) {
    ALLOC(p->dbl.list, m);
    ALLOC(p->dbl.cj, m);
    ALLOC(p->dbl.ck, m);
    ALLOC(p->dbl.aj, m);
    ALLOC(p->dbl.ak, m);
    ALLOC(p->dbl.b, m);
    ALLOC(p->dbl.row_claim, m);
    ALLOC(p->dbl.col_claim, n);
    ALLOC(p->dbl.col_mod, n);
    ALLOC(p->dbl.by, n);
    ALLOC(p->dbl.tb, n);
    ALLOC(p->dbl.total, 2);
    ALLOC(p->dbl.long_task, doubleton_long_cap(N));
    ALLOC(p->dbl.long_cnt, 1);
    ALLOC(p->cp0, n + 1);
    ALLOC(p->ri0, N);
    ALLOC(p->cva0, N);
  }
  if (p->s.enable_dominated) {
    ALLOC(p->dom.ykey, 2 * m);
    ALLOC(p->dom.side, n);
    ALLOC(p->dom.lp_flag, K);
    ALLOC(p->dom.total, 1);
  }
  if (p->s.enable_parallel_cols) {
    ALLOC(p->pc.key, n);
    ALLOC(p->pc.keys, n);
    ALLOC(p->pc.keys2, n);
    ALLOC(p->pc.vals, n);
    ALLOC(p->pc.vals2, n);
    ALLOC(p->pc.lead, n);
    ALLOC(p->pc.lam, n);
    ALLOC(p->pc.nb, n);
    ALLOC(p->pc.terms, n);
    ALLOC(p->pc.total, 1);
  }

  // compaction
  ALLOC(p->cmp.row_new, m + 1);
  ALLOC(p->cmp.col_new, n + 1);
  ALLOC(p->cmp.col_keep, n);
  ALLOC(p->cmp.rbits, m / 64 + 1);
  ALLOC(p->cmp.cbits, n / 64 + 1);
  ALLOC(p->cmp.terms, n);
  ALLOC(p->cmp.pws, pairwise_ws_doubles(n) + 2);
  ALLOC(p->cmp.totals, 4);
  ALLOC(p->cmp.offset, K);
  ALLOC(p->lpr, K + 1);
  p->cmp.ws = p->ws;
  p->cmp.eflag = p->isc.v0;
  p->cmp.qflag = p->isc.v1;
  p->cmp.rowid1 = p->isc.rowid1;
  p->cmp.lpr = p->lpr;
  p->cmp.seg = nullptr;
  p->cmp.seg_host = nullptr;
  p->cmp.lp_off_in = nullptr;

  Reduced& r = p->red;
  ALLOC(r.row_ptr, m + K);
  ALLOC(r.col_idx, N);
  ALLOC(r.val, N);
  ALLOC(r.col_ptr, n + K);
  ALLOC(r.row_idx, N);
  ALLOC(r.cval, N);
  ALLOC(r.lhs, m);
  ALLOC(r.rhs, m);
  ALLOC(r.lb, n);
  ALLOC(r.ub, n);
  ALLOC(r.c, n);
  ALLOC(r.row_map, m);
  ALLOC(r.col_map, n);
  ALLOC(r.row_class, m);
  ALLOC(r.col_class, n);

  // postsolve records: room for one record per row and two per column and
  // some; grown in a run when needed (in static-scratch mode: the rest of
  // the scratch, and a run needing more fails with PSL_ERR_CAPACITY); a
  // fixed stack of device_records records when that is set (flushed)
  p->rec_cap = p->s.device_records > 0 ? p->s.device_records : 2 * m + 4 * n + 1024;
  if (p->carve) {
    int64_t rest = (int64_t)((p->carve_cap - p->carve_used) / sizeof(Record));
    if (rest > p->rec_cap) p->rec_cap = rest;
  }
  ALLOC(p->rec, p->rec_cap);

  HALLOC(p->hflags, 1);
  HALLOC(p->htot, 64);
  HALLOC(p->hoff, 1);
  HALLOC(p->h_lpr, K + 1);
  if (!p->borrowed_events)
    for (auto& e : p->ev) HIPCHK(p, hipEventCreate(&e));

  if (K > 1) {
    ALLOC(p->row_lp, m);
    ALLOC(p->col_lp, n);
    ALLOC(p->lp_row0, K + 1);
    ALLOC(p->lp_col0, K + 1);
    ALLOC(p->lp_round, K);
    ALLOC(p->lp_ok, K);
    ALLOC(p->lpf, K);
    ALLOC(p->lpo, K);
    ALLOC(p->lpt, K);
    ALLOC(p->lp_z0, K + 1);
    ALLOC(p->descs, K);
    ALLOC(p->lp_off_in, K);
    ALLOC(p->rec_off, K + 1);
    ALLOC(p->bins_0, m);
    HALLOC(p->h_row0, K + 1);
    HALLOC(p->h_col0, K + 1);
    HALLOC(p->h_z0, K + 1);
    HALLOC(p->h_round, K);
    HALLOC(p->h_ok, K);
    HALLOC(p->h_lpf, K);
    HALLOC(p->h_lpo, K);
    HALLOC(p->h_lpt, K);
    HALLOC(p->h_desc, K);
    HALLOC(p->h_off_in, K);
    HALLOC(p->h_off, K);
    p->par.lpt = p->lpt;
    p->cmp.seg = p->lp_col0;
    p->cmp.seg_host = p->h_col0;
    p->cmp.lp_off_in = p->lp_off_in;
  }

  d.rp = rp;
  d.ci = ci;
  d.va = va;
  d.cp = cp;
  d.ri = ri;
  d.cva = cva;
  d.lhs = lhs;
  d.rhs = rhs;
  d.bnd = bnd;
  d.bkey = bkey;
  d.src = src;
  d.c = p->c_work;
  d.col_len = col_len;
  d.row_on = row_on;
  d.row_code = row_code;
  d.col_code = col_code;
  d.row_out = row_out;
  d.cand = cand;
  d.chunks0 = p->chunks_0;
  d.cand_cnt = p->cand_cnt;
  d.flags = flags;
  d.cnt = cnt;
  d.off = off;
  d.rec = p->rec;
  d.bins = p->bins_a;
  d.lchunk = p->chunks_a;
  d.dirty = dirty;
  d.rowid1 = p->isc.rowid1;
  d.lpart = lpart;
  d.lrow = lrow;
  d.nlong = 0;
  d.nchunks = 0;
  d.K = 1;
  d.row_lp = p->row_lp;
  d.col_lp = p->col_lp;
  d.lp_row0 = p->lp_row0;
  d.lp_col0 = p->lp_col0;
  d.lp_ok = p->lp_ok;
  d.lp_round = p->lp_round;
  d.lpf = p->lpf;
  d.lpo = p->lpo;
  const psl_settings& s = p->s;
  d.cfg = Cfg{s.feas_tol, s.fix_tol, s.min_improve, s.par_tol, s.inf_value, s.coef_tol, s.enable_dual_fix,
              s.enable_free_singletons, s.enable_forcing_rows};
  // every device array the kernels index must exist (allocations are >= 64 B
  // even for empty problems); colid is set once the transposed copy exists
  const void* ptrs[] = {d.rp, d.ci, d.va, d.cp, d.ri, d.cva, d.lhs, d.rhs, d.bnd, d.bkey, d.src, d.c, d.locks,
                        d.lsrc, d.usrc, d.fs_flag, d.fs_pick, d.owner, d.fs_bad,
                        d.col_len, d.row_on, d.row_code, d.col_code, d.dirty, d.row_out, d.cand, d.cand_cnt,
                        d.flags, d.cnt, d.off, d.rec, d.bins, d.lchunk, d.lpart, d.lrow, p->lpr,
                        d.dense_cols, d.n_dense, d.touch, d.rinf, d.chunks0, d.dirty_tile};
  for (const void* q : ptrs)
    if (!q) return fail(p, PSL_ERR_DEVICE, "internal: a device array was not set up");
  if (K > 1) {
    const void* bp[] = {d.row_lp, d.col_lp, d.lp_row0, d.lp_col0, d.lp_ok, d.lp_round, d.lpf, d.lpo, p->lpt,
                        p->lp_z0, p->descs, p->lp_off_in, p->rec_off, p->bins_0};
    for (const void* q : bp)
      if (!q) return fail(p, PSL_ERR_DEVICE, "internal: a batch array was not set up");
  }
  return PSL_OK;
}

static psl_status read_flags(psl_presolver* p) {
  HIPCHK(p, hipMemcpyAsync(p->hflags, p->d.flags, sizeof(Flags), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return PSL_OK;
}


// workgroups per bin from the current bin offsets and chunk count
static void set_grid(psl_presolver* p) {
  const Dev& d = p->d;
  auto cnt = [&](int b) { return d.bin_off[b + 1] - d.bin_off[b]; };
  for (int b = 0; b < BIN_LONG; ++b) {
    int per_wg = bin_rows(b) * bin_rep(b);  // rows one workgroup sweeps
    p->grid.nb[b] = (cnt(b) + per_wg - 1) / per_wg;
  }
  p->grid.nb[BIN_LONG] = d.nchunks;
  p->grid.long_base = 0;
  for (int b = 0; b < BIN_LONG; ++b) p->grid.long_base += (int64_t)p->grid.nb[b] * cand_region(b);
}

// sweep the rows of view v from now on
static void use_view(psl_presolver* p, const View& v) {
  Dev& d = p->d;
  d.bins = v.bins;
  d.lchunk = v.chunks;
  for (int b = 0; b <= NBINS; ++b) d.bin_off[b] = v.off[b];
  d.nchunks = v.nchunks;
  set_grid(p);
  p->cur = v;
}

// the view described by a selection's device totals (bin offsets, rows,
// nonzeros, chunks)
static View view_of(BinEnt* bins, LongChunk* chunks, const int32_t* tot) {
  View v;
  v.bins = bins;
  v.chunks = chunks;
  for (int b = 0; b <= NBINS; ++b) v.off[b] = tot[b];
  v.rows = tot[NBINS + 1];
  v.nnz = tot[NBINS + 2];
  v.nchunks = tot[NBINS + 3];
  return v;
}

// every active row of an LP still presolving (lp_ok), read back at once
static psl_status full_view(psl_presolver* p, View& dst) {
  Dev& d = p->d;
  select_rows(d, nullptr, 0, p->thresholds[0], p->thresholds[2], p->sel_keep, p->sel_cnt, p->bins_a, p->chunks_a,
              p->sel_dev, p->ws, p->stream);
  HIPCHK(p, hipMemcpyAsync(p->htot, p->sel_dev, (NBINS + 4) * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  dst = view_of(p->bins_a, p->chunks_a, p->htot);
  return PSL_OK;
}

// sweep every active row from now on
static psl_status use_full_view(psl_presolver* p) {
  View v;
  psl_status e = full_view(p, v);
  if (e == PSL_OK) use_view(p, v);
  return e;
}

// queue the next round's selection with the mode the device decided
// (d.flags->mode); read with the round's flags
static void queue_selection(psl_presolver* p) {
  Dev& d = p->d;
  select_rows(d, &d.flags->mode, 0, p->thresholds[0], p->thresholds[2], p->sel_keep, p->sel_cnt, p->bins_s,
              p->chunks_s, d.flags->sel, p->ws, p->stream);
}

static std::string error_what(int32_t bits) {
  if (bits & 1) return "row_ptr must start at 0, be non-decreasing and end at nnz";
  if (bits & 2) return "column index out of range or not strictly ascending within its row";
  if (bits & 4) return "coefficient zero or not finite";
  if (bits & 8) return "side NaN or infinite on the wrong end";
  if (bits & 16) return "bound NaN or infinite on the wrong end";
  return "cost not finite";
}

static std::string error_message(psl_presolver* p, int32_t bits, int64_t pos) {
  if (p->K == 1) {
    p->err_lp = 0;
    return "invalid input: " + error_what(bits) + " (first at index " + std::to_string(pos) + ")";
  }
  // position in the batch's rows, columns or entries -> LP and its own index
  const int64_t* z0 = p->h_z0;
  int k = 0;
  int64_t local = pos;
  auto find = [&](auto start) {
    int lo = 0, hi = p->K - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if ((int64_t)start[mid] <= pos) lo = mid;
      else hi = mid - 1;
    }
    k = lo;
    local = pos - (int64_t)start[lo];
  };
  if (bits & (1 | 8)) find(p->h_row0);
  else if (bits & (2 | 4)) find(z0);
  else find(p->h_col0);
  p->err_lp = k;
  return "invalid input in LP " + std::to_string(k) + ": " + error_what(bits) + " (first at index " +
         std::to_string(local) + ")";
}

// the LP (or union of LPs) of the handle is in d.rp .. p->c_mut; validate,
// transpose, bin
static psl_status ingest_rest(psl_presolver* p) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  int64_t m = p->m, n = p->n, N = p->nnz;
  launch_init_state(d, st);  // clears the flag block
  // the sweep's loads read position 0 for lanes without an entry: with no
  // entries it must still hold a valid column
  if (N == 0) fill_i32((int32_t*)d.ci, 0, 1, st);
  launch_check_rows(d, st);
  check_cols(d, p->lb_in, p->ub_in, p->c_mut, st);
  psl_status s0 = read_flags(p);
  if (s0 != PSL_OK) return s0;
  if (p->hflags->error) return fail(p, PSL_ERR_INVALID, error_message(p, p->hflags->error, p->hflags->error_pos));

  build_rowid(d, p->isc, st);
  launch_check_entries(d, p->isc.rowid1, st);
  s0 = read_flags(p);
  if (s0 != PSL_OK) return s0;
  if (p->hflags->error) return fail(p, PSL_ERR_INVALID, error_message(p, p->hflags->error, p->hflags->error_pos));

  // bins (before the transpose: both use k0/k1); a batch keeps the bins of
  // all its rows apart (the compaction starts from them)
  BinEnt* bins0 = p->K > 1 ? p->bins_0 : p->bins_a;
  LongChunk* chunks0 = p->chunks_0;  // kept intact: the row selections copy from it
  d.bins = bins0;
  d.lchunk = chunks0;
  build_bins(d, p->thresholds, bins0, p->bin_counts_dev, p->isc, st);
  HIPCHK(p, hipMemcpyAsync(p->htot, p->bin_counts_dev, NBINS * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(p, hipStreamSynchronize(st));
  int off = 0;
  for (int b = 0; b < NBINS; ++b) {
    p->bin_counts[b] = p->htot[b];
    d.bin_off[b] = off;
    off += p->htot[b];
  }
  d.bin_off[NBINS] = off;

  // long rows: chunk table built on the device
  int nlong = p->bin_counts[BIN_LONG];
  if (nlong > p->long_cap) return fail(p, PSL_ERR_CAPACITY, "too many long rows");
  d.nlong = nlong;
  build_long_chunks(d, p->thresholds[1] / PASS_LEN, chunks0, d.cnt, d.off, p->bin_counts_dev, p->ws, st);
  HIPCHK(p, hipMemcpyAsync(p->htot, p->bin_counts_dev, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  s0 = read_flags(p);
  if (s0 != PSL_OK) return s0;
  if (p->hflags->error & 64) return fail(p, PSL_ERR_CAPACITY, "a row is longer than 2^26 entries");
  if (p->htot[0] > p->chunk_cap) return fail(p, PSL_ERR_CAPACITY, "too many long-row chunks");
  d.nchunks = p->htot[0];
  d.colid = nullptr;
  View mv;
  mv.bins = bins0;
  mv.chunks = chunks0;
  for (int b = 0; b <= NBINS; ++b) mv.off[b] = d.bin_off[b];
  mv.nchunks = d.nchunks;
  mv.rows = m;
  mv.nnz = N;
  use_view(p, mv);
  if (p->grid.long_base + (int64_t)p->htot[1] > p->cand_cap)
    return fail(p, PSL_ERR_CAPACITY, "candidate buffer too small for the row bins");

  // the reduced problem's value array is free until compaction
  p->colid = build_csc(d, (int32_t*)d.cp, (int32_t*)d.ri, (double*)d.cva, d.col_len, p->isc, p->red.val, st);
  p->cmp.colid = p->colid;
  d.colid = p->colid;
  list_dense_cols(d, st);
  if (p->s.enable_doubletons) {
    // the input's transposed copy for the dual postsolve; no column kept yet
    HIPCHK(p, hipMemcpyAsync(p->cp0, d.cp, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (N) {
      HIPCHK(p, hipMemcpyAsync(p->ri0, d.ri, N * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      HIPCHK(p, hipMemcpyAsync(p->cva0, d.cva, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    launch_doubleton_init(d, p->dbl, st);
  }

  // parallel-row table: one slice of >= 2 m_k slots per LP
  if (p->K == 1) {
    int64_t cap = 64;
    while (cap < 2 * m) cap <<= 1;
    p->par.cap = cap;
  } else {
    int64_t base = 0;
    for (int k = 0; k < p->K; ++k) {
      int64_t mk = p->h_row0[k + 1] - p->h_row0[k], cap = 64;
      while (cap < 2 * mk) cap <<= 1;
      p->h_lpt[k] = LpTab{base, cap};
      base += cap;
    }
    if (base > p->par_slots) return fail(p, PSL_ERR_DEVICE, "internal: parallel-row table too small");
    p->par.cap = base;
    HIPCHK(p, hipMemcpyAsync(p->lpt, p->h_lpt, p->K * sizeof(LpTab), hipMemcpyHostToDevice, st));
  }
  (void)n;
  HIPCHK(p, hipEventRecord(p->ev[1], st));
  HIPCHK(p, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(p, hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
  p->ms_ingest = ms;
  p->state = 0;
  p->host_rec_valid = false;
  return PSL_OK;
}

static void set_sizes(psl_presolver* p, int32_t K, int32_t m, int32_t n, int64_t nnz) {
  p->K = K;
  p->m = m;
  p->n = n;
  p->nnz = nnz;
  p->d.K = K;
  p->d.m = m;
  p->d.n = n;
  p->d.nnz = nnz;
}

// copy + validate + transpose + bins of one LP whose shape equals the handle's
static psl_status ingest(psl_presolver* p, const psl_lp* lp) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  int64_t m = p->m, n = p->n, N = p->nnz;
  HIPCHK(p, hipEventRecord(p->ev[0], st));
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, st);
  };
  HIPCHK(p, cp((void*)d.rp, lp->row_ptr, (m + 1) * 4 * (m > 0)));
  if (m == 0) fill_i32((int32_t*)d.rp, 0, 1, st);
  HIPCHK(p, cp((void*)d.ci, lp->col_idx, N * 4));
  HIPCHK(p, cp((void*)d.va, lp->val, N * 8));
  HIPCHK(p, cp(d.lhs, lp->lhs, m * 8));
  HIPCHK(p, cp(d.rhs, lp->rhs, m * 8));
  HIPCHK(p, cp(p->lb_in, lp->lb, n * 8));
  HIPCHK(p, cp(p->ub_in, lp->ub, n * 8));
  HIPCHK(p, cp(p->c_mut, lp->c, n * 8));
  p->obj_offset = lp->obj_offset == 0.0 ? 0.0 : lp->obj_offset;
  return ingest_rest(p);
}

// a batch of k LPs (shapes already checked to fit): the union goes into the
// handle's arrays, from host memory through host-side packing, from device
// memory by the gather kernels
static psl_status ingest_batch(psl_presolver* p, int32_t k, const psl_lp* lps) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  int64_t M = 0, Nc = 0, Z = 0;
  for (int32_t t = 0; t < k; ++t) {
    p->h_row0[t] = (int32_t)M;
    p->h_col0[t] = (int32_t)Nc;
    p->h_z0[t] = Z;
    p->h_off_in[t] = lps[t].obj_offset == 0.0 ? 0.0 : lps[t].obj_offset;
    M += lps[t].m;
    Nc += lps[t].n;
    Z += lps[t].nnz;
  }
  p->h_row0[k] = (int32_t)M;
  p->h_col0[k] = (int32_t)Nc;
  p->h_z0[k] = Z;
  set_sizes(p, k, (int32_t)M, (int32_t)Nc, Z);
  p->obj_offset = 0.0;
  HIPCHK(p, hipEventRecord(p->ev[0], st));
  HIPCHK(p, hipMemcpyAsync(p->lp_row0, p->h_row0, (k + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(p, hipMemcpyAsync(p->lp_col0, p->h_col0, (k + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(p, hipMemcpyAsync(p->lp_z0, p->h_z0, (k + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(p, hipMemcpyAsync(p->lp_off_in, p->h_off_in, k * sizeof(double), hipMemcpyHostToDevice, st));
  launch_init_state(d, st);  // clears the error flags for the gather's checks
  if (lps[0].mem == PSL_MEM_DEVICE) {
    for (int32_t t = 0; t < k; ++t) {
      const psl_lp& L = lps[t];
      p->h_desc[t] = LpDesc{L.row_ptr, L.col_idx, L.val, L.lhs, L.rhs, L.lb, L.ub, L.c, L.m, L.n, L.nnz};
    }
    HIPCHK(p, hipMemcpyAsync(p->descs, p->h_desc, k * sizeof(LpDesc), hipMemcpyHostToDevice, st));
    batch_gather(d, p->descs, p->lp_z0, (int32_t*)d.rp, (int32_t*)d.ci, (double*)d.va, d.lhs, d.rhs, p->lb_in,
                 p->ub_in, p->c_mut, p->row_lp, p->col_lp, st);
    fill_i32((int32_t*)d.rp + M, (int32_t)Z, 1, st);
  } else {
    // host: pack the union (row pointers and column indices shifted)
    std::vector<int32_t> rp(M + 1), ci(Z);
    std::vector<double> va(Z), lhs(M), rhs(M), lb(Nc), ub(Nc), c(Nc);
    for (int32_t t = 0; t < k; ++t) {
      const psl_lp& L = lps[t];
      int64_t r0 = p->h_row0[t], c0 = p->h_col0[t], z0 = p->h_z0[t];
      if (L.m > 0 && (L.row_ptr[0] != 0 || (int64_t)L.row_ptr[L.m] != L.nnz)) {
        p->err_lp = t;
        return fail(p, PSL_ERR_INVALID, "invalid input in LP " + std::to_string(t) + ": " + error_what(1));
      }
      for (int32_t i = 0; i < L.m; ++i) rp[r0 + i] = (int32_t)(L.row_ptr[i] + z0);
      for (int64_t q = 0; q < L.nnz; ++q) {
        int32_t j = L.col_idx[q];
        if (j < 0 || j >= L.n) {
          p->err_lp = t;
          return fail(p, PSL_ERR_INVALID, "invalid input in LP " + std::to_string(t) + ": " + error_what(2) +
                                              " (first at index " + std::to_string(q) + ")");
        }
        ci[z0 + q] = (int32_t)(j + c0);
      }
      if (L.nnz) std::memcpy(&va[z0], L.val, L.nnz * sizeof(double));
      if (L.m) {
        std::memcpy(&lhs[r0], L.lhs, L.m * sizeof(double));
        std::memcpy(&rhs[r0], L.rhs, L.m * sizeof(double));
      }
      if (L.n) {
        std::memcpy(&lb[c0], L.lb, L.n * sizeof(double));
        std::memcpy(&ub[c0], L.ub, L.n * sizeof(double));
        std::memcpy(&c[c0], L.c, L.n * sizeof(double));
      }
    }
    rp[M] = (int32_t)Z;
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
      if (bytes == 0) return hipSuccess;
      return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    HIPCHK(p, hipStreamSynchronize(st));
    HIPCHK(p, up((void*)d.rp, rp.data(), (M + 1) * 4));
    HIPCHK(p, up((void*)d.ci, ci.data(), Z * 4));
    HIPCHK(p, up((void*)d.va, va.data(), Z * 8));
    HIPCHK(p, up(d.lhs, lhs.data(), M * 8));
    HIPCHK(p, up(d.rhs, rhs.data(), M * 8));
    HIPCHK(p, up(p->lb_in, lb.data(), Nc * 8));
    HIPCHK(p, up(p->ub_in, ub.data(), Nc * 8));
    HIPCHK(p, up(p->c_mut, c.data(), Nc * 8));
    batch_maps(d, p->row_lp, p->col_lp, st);
  }
  psl_status s0 = read_flags(p);
  if (s0 != PSL_OK) return s0;
  if (p->hflags->error) return fail(p, PSL_ERR_INVALID, error_message(p, p->hflags->error, p->hflags->error_pos));
  return ingest_rest(p);
}

// settings of a new handle (thresholds copied, the caller's array not kept)
static void take_settings(psl_presolver* p, const psl_settings* s) {
  p->s = *s;
  p->s.bin_thresholds = nullptr;
  if (s->bin_thresholds) {
    p->thresholds[0] = s->bin_thresholds[0];
    p->thresholds[1] = s->bin_thresholds[1];
    if (s->n_bins == 3) p->thresholds[2] = s->bin_thresholds[2];
  }
  p->stream = (hipStream_t)s->stream;
  p->sweep_mode = s->split_sweep ? 2 : MODE_ROUND;
  if (const char* e = std::getenv("PSL_TRACE")) p->trace = std::atoi(e) != 0;
}

// records one phase may add: a round (a row record per row, two bound changes
// and a fixing per column) or a parallel pass (a record per row and column for
// the parallel rows and columns, one per column for dominated columns, and
// for doubletons one per row and two per column)
static int64_t pass_records(const psl_settings* s, int64_t m, int64_t n) {
  return m + n + (s->enable_dominated ? n : 0) + (s->enable_doubletons ? m + 2 * n : 0) + 16;
}

static int64_t phase_records(const psl_settings* s, int64_t m, int64_t n) {
  return std::max(m + 3 * n + 16, pass_records(s, m, n));
}

extern "C" psl_status psl_presolve_create(const psl_lp* lp, const psl_settings* s, psl_presolver** out) {
  if (!lp || !out) {
    g_create_error = "null argument";
    return PSL_ERR_INVALID;
  }
  psl_settings def;
  psl_settings_default(&def);
  if (!s) s = &def;
  std::string e = check_settings(s);
  if (e.empty()) e = check_lp_shape(lp);
  if (e.empty() && s->device_records > 0 && s->device_records < phase_records(s, lp->m, lp->n))
    e = "device_records must hold one phase's records: at least " + std::to_string(phase_records(s, lp->m, lp->n));
  if (!e.empty()) {
    g_create_error = e;
    return PSL_ERR_INVALID;
  }
  if (hipSetDevice(s->device) != hipSuccess) {
    g_create_error = "cannot select the device";
    return PSL_ERR_DEVICE;
  }
  psl_presolver* p = new psl_presolver();
  take_settings(p, s);
  p->cap_m = lp->m;
  p->cap_n = lp->n;
  p->cap_nnz = lp->nnz;
  p->cap_K = 1;
  set_sizes(p, 1, lp->m, lp->n, lp->nnz);
  psl_status st = setup_arena(p);
  if (st == PSL_OK) st = ingest(p, lp);
  if (st != PSL_OK) {
    g_create_error = p->err;
    psl_presolve_free(p);
    return st;
  }
  *out = p;
  return PSL_OK;
}

extern "C" psl_status psl_presolve_reload(psl_presolver* p, const psl_lp* lp) {
  if (!p || !lp) return PSL_ERR_INVALID;
  std::string e = check_lp_shape(lp);
  if (!e.empty()) return fail(p, PSL_ERR_INVALID, e);
  if (p->cap_K != 1 || lp->m != p->cap_m || lp->n != p->cap_n || lp->nnz != p->cap_nnz)
    return fail(p, PSL_ERR_INVALID, "reload needs the same m, n and nnz");
  if (hipSetDevice(p->s.device) != hipSuccess) return fail(p, PSL_ERR_DEVICE, "cannot select the device");
  psl_status st = ingest(p, lp);
  if (st != PSL_OK) p->state = 2;  // unusable until a successful reload
  return st;
}

// Room for `need` more records on the device: a fixed stack (device_records
// > 0) is flushed to host memory and emptied; otherwise the buffer grows.
static psl_status ensure_capacity(psl_presolver* p, int64_t need) {
  int64_t used = p->rec_count - p->rec_flushed;
  if (used + need <= p->rec_cap) return PSL_OK;
  if (p->s.device_records > 0) {
    if (need > p->rec_cap) return fail(p, PSL_ERR_CAPACITY, "a phase's records exceed device_records");
    size_t at = p->flushed.size();
    p->flushed.resize(at + (size_t)used);
    HIPCHK(p, hipMemcpyAsync(p->flushed.data() + at, p->rec, used * sizeof(Record), hipMemcpyDeviceToHost,
                             p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    p->rec_flushed = p->rec_count;
    p->flushes += 1;
    return PSL_OK;
  }
  if (p->carve) return fail(p, PSL_ERR_CAPACITY, "the postsolve records outgrow the static scratch");
  int64_t cap = std::max<int64_t>(2 * p->rec_cap, p->rec_count + need + 1024);
  Record* nr = nullptr;
  psl_status st = dalloc(p, &nr, cap);
  if (st != PSL_OK) return st;
  if (p->rec_count)
    HIPCHK(p, hipMemcpyAsync(nr, p->rec, p->rec_count * sizeof(Record), hipMemcpyDeviceToDevice, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  auto it = std::find(p->allocs.begin(), p->allocs.end(), (void*)p->rec);
  if (it != p->allocs.end()) {
    (void)hipFree(p->rec);
    p->allocs.erase(it);
  }
  p->rec = nr;
  p->d.rec = nr;
  p->rec_cap = cap;
  return PSL_OK;
}

static float elapsed(psl_presolver* p, int a, int b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, p->ev[a], p->ev[b]) != hipSuccess) return 0.f;
  return ms;
}

// K > 1: upload the LPs' round numbers and clear their flags before a round
static psl_status begin_lp_round(psl_presolver* p) {
  if (p->K == 1) return PSL_OK;
  HIPCHK(p, hipMemcpyAsync(p->lp_round, p->h_round, p->K * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipMemsetAsync(p->lpf, 0, p->K * sizeof(LpFlags), p->stream));
  HIPCHK(p, hipMemsetAsync(p->lpo, 0, p->K * sizeof(LpOut), p->stream));
  return PSL_OK;
}

// K > 1: queue the readback of the LPs' flags (and record counts); the next
// synchronising read completes it
static psl_status queue_lp_read(psl_presolver* p, bool totals) {
  if (p->K == 1) return PSL_OK;
  if (totals) HIPCHK(p, hipMemcpyAsync(p->h_lpo, p->lpo, p->K * sizeof(LpOut), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipMemcpyAsync(p->h_lpf, p->lpf, p->K * sizeof(LpFlags), hipMemcpyDeviceToHost, p->stream));
  return PSL_OK;
}

// K > 1: LPs that stopped leave the row selections (the device clears
// lp_ok itself for an LP found infeasible or unbounded)
static psl_status drop_done_lps(psl_presolver* p) {
  for (int k = 0; k < p->K; ++k) p->h_ok[k] = p->lst[k].phase != LP_DONE;
  HIPCHK(p, hipMemcpyAsync(p->lp_ok, p->h_ok, p->K, hipMemcpyHostToDevice, p->stream));
  return PSL_OK;
}

// scratch of the record split (K > 1), grown to the record count
static psl_status split_records(psl_presolver* p) {
  int64_t cnt = p->rec_count;
  if (cnt > p->split_cap) {
    for (void* q : {(void*)p->rec_lp, (void*)p->sk0, (void*)p->sk1, (void*)p->sv0, (void*)p->sv1, (void*)p->sws}) {
      auto it = std::find(p->allocs.begin(), p->allocs.end(), q);
      if (q && it != p->allocs.end()) {
        (void)hipFree(q);
        p->allocs.erase(it);
      }
    }
    int64_t cap = std::max<int64_t>(cnt, 1024);
    ALLOC(p->rec_lp, cap);
    ALLOC(p->sk0, cap);
    ALLOC(p->sk1, cap);
    ALLOC(p->sv0, cap);
    ALLOC(p->sv1, cap);
    ALLOC(p->sws, rec_split_ws_ints(cap) + 64);
    p->split_cap = cap;
  }
  rec_split(p->d, p->rec, cnt, p->rec_lp, p->rec_off, p->sk0, p->sk1, p->sv0, p->sv1, p->sws, p->stream);
  p->h_rec_off.resize(p->K + 1);
  HIPCHK(p, hipMemcpyAsync(p->h_rec_off.data(), p->rec_off, (p->K + 1) * sizeof(int32_t), hipMemcpyDeviceToHost,
                           p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return PSL_OK;
}

// The round controller for K >= 1 LPs. Each LP's life, as for one LP alone:
// round 0 (input fixings); then outer cycles of propagation rounds until a
// round changes nothing or max_rounds is reached, followed by a parallel-row
// pass, another cycle only if that pass merged rows; infeasible or unbounded
// ends it at once. In a batch an LP that converged waits for the cycle's
// parallel pass (sweeping its rows again changes nothing); LPs that stopped
// are dropped from the bin lists. The run goes unit by unit (EngRun): each
// launch queues a unit's kernels and the reads of its results, each
// completion waits for them and decides the next unit.

static bool lp_inf(const psl_presolver* p, int k) {
  return p->K > 1 ? p->h_lpf[k].infeasible != 0 : p->hflags->infeasible != 0;
}
static bool lp_unb(const psl_presolver* p, int k) {
  return p->K > 1 ? p->h_lpf[k].unbounded != 0 : p->hflags->unbounded != 0;
}
static bool lp_merged(const psl_presolver* p, int k) {
  return p->K > 1 ? p->h_lpf[k].merged != 0 : p->hflags->merged != 0;
}
static int32_t lp_total(const psl_presolver* p, int k) {
  return p->K > 1 ? p->h_lpo[k].total : p->hflags->round_total;
}

// queue the read of the device flags (completed by the unit's wait)
static psl_status queue_flags(psl_presolver* p) {
  HIPCHK(p, hipMemcpyAsync(p->hflags, p->d.flags, sizeof(Flags), hipMemcpyDeviceToHost, p->stream));
  return PSL_OK;
}

psl_status psl::engine_start(psl_presolver* p) {
  if (p->state != 0) return fail(p, PSL_ERR_STATE, "run needs a fresh load");
  const int K = p->K;
  p->rec_count = 0;
  p->rec_flushed = 0;
  p->flushes = 0;
  p->flushed.clear();
  p->host_rec_valid = false;
  p->lp_host_rec.clear();
  p->state = 1;
  p->lst.assign(K, LpState{});
  p->run = EngRun{};
  p->run.S.nnz_in = p->nnz;
  p->run.unit = U_ROUND0;
  HIPCHK(p, hipEventRecord(p->ev[2], p->stream));
  if (K > 1) {
    for (int k = 0; k < K; ++k) {
      p->h_ok[k] = 1;
      p->h_round[k] = 0;
    }
    HIPCHK(p, hipMemcpyAsync(p->lp_ok, p->h_ok, K, hipMemcpyHostToDevice, p->stream));
    psl_status e0 = begin_lp_round(p);
    if (e0 != PSL_OK) return e0;
  }
  return PSL_OK;
}

// the top of an outer cycle: its first round, or the compaction when no LP
// propagates any more
static psl_status cycle_start(psl_presolver* p) {
  EngRun& R = p->run;
  int nprop = 0;
  if (R.outer < p->s.max_outer)
    for (auto& L : p->lst)
      if (L.phase == LP_PROP) {
        L.cycles = R.outer + 1;
        ++nprop;
      }
  if (nprop == 0) {
    R.unit = U_COMPACT;
    return PSL_OK;
  }
  R.consts_current = false;
  R.r = 0;
  R.unit = U_ROUND;
  // a cycle's first round sweeps every active row
  return use_full_view(p);
}

// after a cycle's rounds: its reduction pass, or the compaction
static void rounds_end(psl_presolver* p) {
  const psl_settings& s = p->s;
  int npar = 0;
  for (auto& L : p->lst)
    if (L.phase != LP_DONE) ++npar;
  if (npar == 0) {
    p->run.unit = U_COMPACT;
    return;
  }
  if (!s.enable_parallel_rows && !s.enable_parallel_cols && !s.enable_doubletons && !s.enable_dominated) {
    for (auto& L : p->lst) L.phase = LP_DONE;
    p->run.unit = U_COMPACT;
    return;
  }
  p->run.unit = U_PASS;
}

static psl_status launch_round0(psl_presolver* p) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  int64_t m = p->m, n = p->n;
  // the run works on a copy of the costs (free-singleton substitutions
  // change it); the input's stay for postsolve
  if (n) HIPCHK(p, hipMemcpyAsync(p->c_work, p->c_mut, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  // round 0: input fixings
  launch_init_state(d, st);
  launch_round0_count(d, st);
  scan_excl(d.cnt, d.off, m + n, &d.flags->round_total, p->ws, st);
  launch_round0_emit(d, 0, st);
  if (p->s.enable_dual_fix) init_locks(d, p->isc.v0, p->isc.v1, p->ws, st);  // ingest scratch, free until compaction
  psl_status e = queue_lp_read(p, false);
  if (e != PSL_OK) return e;
  return queue_flags(p);
}

static psl_status complete_round0(psl_presolver* p) {
  p->rec_count += p->hflags->round_total;
  bool any_done = false;
  for (int k = 0; k < p->K; ++k)
    if (lp_inf(p, k)) {
      p->lst[k].phase = LP_DONE;
      p->lst[k].infeasible = true;
      p->lst[k].cycles = 1;
      any_done = true;
    }
  if (p->K > 1 && any_done) {
    psl_status e = drop_done_lps(p);
    if (e != PSL_OK) return e;
  }
  return cycle_start(p);
}

static psl_status launch_round(psl_presolver* p) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  const psl_settings& s = p->s;
  EngRun& R = p->run;
  int64_t m = p->m, n = p->n;
  ++R.round;
  for (int k = 0; k < p->K; ++k)
    if (p->lst[k].phase == LP_PROP) {
      ++p->lst[k].rounds;
      if (p->K > 1) p->h_round[k] = p->lst[k].rounds;
    }
  psl_status e = ensure_capacity(p, m + 3 * n + 16);
  if (e == PSL_OK) e = begin_lp_round(p);
  if (e != PSL_OK) return e;
  HIPCHK(p, hipEventRecord(p->ev[4], st));
  launch_long_stats(d, MODE_ROUND, st);
  HIPCHK(p, hipEventRecord(p->ev[7], st));
  launch_sweep(d, p->grid, p->sweep_mode, st);
  HIPCHK(p, hipEventRecord(p->ev[5], st));
  launch_src(d, p->grid, st);
  launch_decide(d, p->rec_count - p->rec_flushed, R.round, d.cnt, d.off, p->ws, st);
  // (the candidate regions are free until the next sweep)
  if (s.enable_free_singletons)
    launch_free_singletons(d, reinterpret_cast<int32_t*>(d.cand), p->rec_count - p->rec_flushed, R.round, p->ws,
                           st);
  HIPCHK(p, hipEventRecord(p->ev[6], st));
  // The next round's selection is made before the round's one read, in
  // one pass over the rows. Rows none of whose columns changed since they
  // were last swept give the same statistics and no qualifying candidate,
  // so after a round with few column changes only the touched (marked)
  // rows are swept; and inert rows (their infinite-contribution counts,
  // kept current as bounds become finite, rule out every outcome) are
  // never swept. The counts are kept by decrements while few bounds
  // become finite in a round. After a round with many, no decrement is
  // made and the next round skips no row: it sweeps, and so recounts,
  // every row one of whose bounds became finite, while the counts of the
  // rows it does not sweep are still exact; after it the counts are
  // exact again. The device takes these decisions from the round's totals
  // (d.flags->mode); an LP that stopped has left lp_ok already. When the
  // rounds end here the selection is not used.
  if (!d.dirty || !d.colid) return fail(p, PSL_ERR_DEVICE, "internal: incremental state not set up");
  mark_dirty(d, R.r + 1 < s.max_rounds, p->incr_factor, p->count_factor, st);
  queue_selection(p);
  e = queue_lp_read(p, true);
  if (e != PSL_OK) return e;
  return queue_flags(p);
}

static psl_status complete_round(psl_presolver* p) {
  EngRun& R = p->run;
  psl_stats& S = R.S;
  int64_t m = p->m, n = p->n;
  int32_t removed = p->hflags->rows_removed;
  R.long_ms += elapsed(p, 4, 7);
  R.sweep_ms += elapsed(p, 7, 5);
  R.decide_ms += elapsed(p, 5, 6);
  S.sweep_launches += 1;
  S.sweep_nnz += p->cur.nnz;
  // algorithmic bytes of the sweep launch: the swept rows' positions
  // (12 B a nonzero); per swept row its bin entry, row pointer, sides and
  // statistics (48 B); per column it can touch (at most one per nonzero)
  // the bound read and the new-bound write (32 B)
  {
    double sb = 12.0 * p->cur.nnz + 48.0 * p->cur.rows + 32.0 * std::min<int64_t>(n, p->cur.nnz);
    S.sweep_bytes += sb;
    // the decisions over every row and column, and the round's records
    S.alg_bytes += sb + 40.0 * ((double)m + n) + 48.0 * p->hflags->round_total;
  }
  p->rec_count += p->hflags->round_total;
  bool any_done = false;
  int nprop = 0;
  for (int k = 0; k < p->K; ++k) {
    LpState& L = p->lst[k];
    if (L.phase != LP_PROP) continue;
    if (lp_inf(p, k)) {
      L.phase = LP_DONE;
      L.infeasible = true;
      any_done = true;
    } else if (lp_unb(p, k)) {
      L.phase = LP_DONE;
      L.unbounded = true;
      any_done = true;
    } else if (lp_total(p, k) == 0) {
      L.phase = LP_WAIT;
    } else {
      ++nprop;
    }
  }
  if (p->trace)
    std::fprintf(stderr, "[psl] round %d: swept rows %lld nnz %lld, records %d, rows removed %d, "
                 "bounds made finite %d, LPs propagating %d\n", R.round, (long long)p->cur.rows,
                 (long long)p->cur.nnz, p->hflags->round_total, removed, p->hflags->fin_cols, nprop);
  if (nprop == 0) {
    rounds_end(p);
    return PSL_OK;
  }
  if (p->K > 1 && any_done) {
    psl_status e = drop_done_lps(p);
    if (e != PSL_OK) return e;
  }
  use_view(p, view_of(p->bins_s, p->chunks_s, p->hflags->sel));
  if (++R.r < p->s.max_rounds) R.unit = U_ROUND;
  else rounds_end(p);
  return PSL_OK;
}

// the cycle's reduction pass (parallel rows, then the optional column
// explorers), for every LP still presolving
static psl_status launch_pass(psl_presolver* p) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  const psl_settings& s = p->s;
  EngRun& R = p->run;
  int64_t m = p->m, n = p->n;
  ++R.round;
  for (int k = 0; k < p->K; ++k)
    if (p->lst[k].phase != LP_DONE) {
      ++p->lst[k].rounds;
      if (p->K > 1) p->h_round[k] = p->lst[k].rounds;
    }
  psl_status e = use_full_view(p);
  // row records, then column records (and a substitution pass's)
  if (e == PSL_OK) e = ensure_capacity(p, pass_records(&s, m, n));
  if (e == PSL_OK) e = begin_lp_round(p);
  if (e != PSL_OK) return e;
  HIPCHK(p, hipEventRecord(p->ev[4], st));
  // every live row's removed-column constant and active length go to
  // row_out (free once the round's records are emitted): long rows from
  // their chunk partials here, the others in the hash pass
  if (s.enable_parallel_rows) launch_long_consts(d, st);
  launch_par_reset(d, p->par, st);
  if (s.enable_parallel_rows) {
    launch_par_hash(d, p->par, p->grid, st);
    launch_par_verify(d, p->par, st);
    launch_par_count(d, p->par, st);
    scan_excl(d.cnt, d.off, m, &d.flags->round_total, p->ws, st);
    launch_par_emit(d, p->par, p->rec_count - p->rec_flushed, R.round, st);
    launch_par_drop(d, p->par, st);
  } else {
    fill_i32(&d.flags->round_total, 0, 1, st);
  }
  // parallel columns on the rows the row pass left (an LP it found
  // infeasible has stopped)
  if (s.enable_parallel_cols) launch_par_cols(d, p->pc, p->rec_count - p->rec_flushed, R.round, p->ws, st);
  if (s.enable_dominated) launch_dominated(d, p->dom, p->rec_count - p->rec_flushed, R.round, p->ws, st);
  if (s.enable_doubletons) {
    // active lengths and removed-column constants after the parallel
    // passes (row_out), then the substitutions
    launch_long_stats(d, MODE_COMPACT, st);
    launch_sweep(d, p->grid, MODE_COMPACT, st);
    launch_doubletons(d, p->dbl, p->rec_count - p->rec_flushed, R.round, p->ws, st);
  }
  HIPCHK(p, hipEventRecord(p->ev[5], st));
  e = queue_lp_read(p, false);
  if (e != PSL_OK) return e;
  return queue_flags(p);
}

static psl_status complete_pass(psl_presolver* p) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  const psl_settings& s = p->s;
  EngRun& R = p->run;
  psl_stats& S = R.S;
  int64_t m = p->m;
  R.consts_current = p->K == 1 && s.enable_parallel_rows && !p->hflags->merged;
  R.par_ms += elapsed(p, 4, 5);
  if (s.enable_doubletons && p->hflags->dbl_applied) {
    // rows were rewritten: the transposed copy (and what hangs on it) again
    p->colid = build_csc(d, (int32_t*)d.cp, (int32_t*)d.ri, (double*)d.cva, d.cnt, p->isc, p->red.val, st);
    p->cmp.colid = p->colid;
    d.colid = p->colid;
    list_dense_cols(d, st);
    launch_doubleton_relock(d, p->dbl, st);
    S.alg_bytes += 36.0 * (double)p->nnz;
  }
  // keys and table per row, one pass over the positions, the records
  S.alg_bytes += 40.0 * m + 12.0 * (double)p->nnz + 48.0 * p->hflags->round_total;
  p->rec_count += p->hflags->round_total;
  bool any_done = false;
  for (int k = 0; k < p->K; ++k) {
    LpState& L = p->lst[k];
    if (L.phase == LP_DONE) continue;
    if (lp_inf(p, k)) {
      L.phase = LP_DONE;
      L.infeasible = true;
    } else if (lp_unb(p, k)) {  // dominated columns: an infinite fixing or crossing dual bounds
      L.phase = LP_DONE;
      L.unbounded = true;
    } else if (lp_merged(p, k) && R.outer + 1 < s.max_outer) {
      L.phase = LP_PROP;
    } else {
      L.phase = LP_DONE;
    }
    any_done |= L.phase == LP_DONE;
  }
  if (p->K > 1 && any_done) {
    psl_status e = drop_done_lps(p);
    if (e != PSL_OK) return e;
  }
  ++R.outer;
  return cycle_start(p);
}

// compaction of the LPs that ended feasible
static psl_status launch_compact(psl_presolver* p) {
  Dev& d = p->d;
  hipStream_t st = p->stream;
  EngRun& R = p->run;
  const int K = p->K;
  R.any_feasible = false;
  for (auto& L : p->lst) R.any_feasible |= !L.infeasible && !L.unbounded;
  p->red_m = p->red_n = 0;
  p->red_nnz = 0;
  if (!R.any_feasible) return PSL_OK;
  if (K > 1) {
    for (int k = 0; k < K; ++k) p->h_ok[k] = !p->lst[k].infeasible && !p->lst[k].unbounded;
    HIPCHK(p, hipMemcpyAsync(p->lp_ok, p->h_ok, K, hipMemcpyHostToDevice, st));
  }
  psl_status e = use_full_view(p);
  if (e != PSL_OK) return e;
  HIPCHK(p, hipEventRecord(p->ev[4], st));
  if (!R.consts_current) {
    launch_long_stats(d, MODE_COMPACT, st);
    launch_sweep(d, p->grid, MODE_COMPACT, st);
  }
  compact_flags(d, p->cmp, st);
  compact_write(d, p->cmp, p->red, p->obj_offset, st);
  HIPCHK(p, hipEventRecord(p->ev[5], st));
  HIPCHK(p, hipMemcpyAsync(p->htot, p->cmp.totals, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(p, hipMemcpyAsync(p->h_lpr, p->lpr, (K + 1) * sizeof(LpRed), hipMemcpyDeviceToHost, st));
  if (K > 1) HIPCHK(p, hipMemcpyAsync(p->h_off, p->cmp.offset, K * sizeof(double), hipMemcpyDeviceToHost, st));
  else HIPCHK(p, hipMemcpyAsync(p->hoff, p->cmp.offset, sizeof(double), hipMemcpyDeviceToHost, st));
  return PSL_OK;
}

static psl_status complete_compact(psl_presolver* p) {
  EngRun& R = p->run;
  psl_stats& S = R.S;
  const int K = p->K;
  const bool B = K > 1;
  if (R.any_feasible) {
    R.cmp_ms = elapsed(p, 4, 5);
    p->red_m = p->htot[0];
    p->red_n = p->htot[1];
    p->red_nnz = p->htot[2];
    p->red_off = B ? 0.0 : *p->hoff;
    S.alg_bytes += 12.0 * (double)p->nnz + 24.0 * (double)p->red_nnz + 32.0 * p->red_m + 40.0 * p->red_n;
    if (p->htot[2] != p->htot[3]) return fail(p, PSL_ERR_DEVICE, "reduced CSR and transposed copy disagree");
    for (int k = 0; k < K; ++k)
      if (p->h_lpr[k + 1].eb - p->h_lpr[k].eb != p->h_lpr[k + 1].qb - p->h_lpr[k].qb)
        return fail(p, PSL_ERR_DEVICE, "reduced CSR and transposed copy disagree");
  }
  if (B) {
    psl_status e = split_records(p);
    if (e != PSL_OK) return e;
  }
  HIPCHK(p, hipEventRecord(p->ev[3], p->stream));
  HIPCHK(p, hipEventSynchronize(p->ev[3]));

  p->lp_result.resize(K);
  for (int k = 0; k < K; ++k) {
    const LpState& L = p->lst[k];
    int64_t recs = B ? p->h_rec_off[k + 1] - p->h_rec_off[k] : p->rec_count;
    p->lp_result[k] = L.infeasible ? PSL_RES_INFEASIBLE
                      : L.unbounded ? PSL_RES_UNBOUNDED_OR_INFEASIBLE
                      : recs ? PSL_RES_REDUCED
                             : PSL_RES_UNCHANGED;
  }
  p->result = p->lp_result[0];
  S.rounds = R.round;
  S.outer_cycles = 1;
  for (auto& L : p->lst) S.outer_cycles = std::max(S.outer_cycles, L.cycles);
  S.records = p->rec_count;
  S.record_flushes = p->flushes;
  S.nnz_out = p->red_nnz;
  S.m_out = p->red_m;
  S.n_out = p->red_n;
  S.ms_ingest = p->ms_ingest;
  S.ingest_bytes = 36.0 * (double)p->nnz + 32.0 * p->m + 48.0 * p->n;
  S.ms_sweep = R.sweep_ms;
  S.ms_long = R.long_ms;
  S.ms_decide = R.decide_ms;
  S.ms_parallel = R.par_ms;
  S.ms_compact = R.cmp_ms;
  S.ms_total = elapsed(p, 2, 3);
  p->stats = S;
  R.unit = U_DONE;
  return PSL_OK;
}

psl_status psl::engine_launch(psl_presolver* p) {
  switch (p->run.unit) {
    case U_ROUND0: return launch_round0(p);
    case U_ROUND: return launch_round(p);
    case U_PASS: return launch_pass(p);
    case U_COMPACT: return launch_compact(p);
    default: return fail(p, PSL_ERR_STATE, "the run has ended");
  }
}

psl_status psl::engine_complete(psl_presolver* p, bool* done) {
  *done = false;
  HIPCHK(p, hipStreamSynchronize(p->stream));
  psl_status e;
  switch (p->run.unit) {
    case U_ROUND0: e = complete_round0(p); break;
    case U_ROUND: e = complete_round(p); break;
    case U_PASS: e = complete_pass(p); break;
    case U_COMPACT: e = complete_compact(p); break;
    default: return fail(p, PSL_ERR_STATE, "the run has ended");
  }
  *done = e == PSL_OK && p->run.unit == U_DONE;
  return e;
}

static psl_status run_engine(psl_presolver* p, psl_stats* out) {
  psl_status e = psl::engine_start(p);
  bool done = false;
  while (e == PSL_OK && !done) {
    e = psl::engine_launch(p);
    if (e == PSL_OK) e = psl::engine_complete(p, &done);
  }
  if (e != PSL_OK) return e;
  if (out) *out = p->stats;
  return PSL_OK;
}

extern "C" psl_status psl_presolve_run(psl_presolver* p, psl_result* res, psl_stats* stats) {
  if (!p || !res) return PSL_ERR_INVALID;
  if (p->state != 0) return fail(p, PSL_ERR_STATE, "run needs a fresh create or reload");
  if (hipSetDevice(p->s.device) != hipSuccess) return fail(p, PSL_ERR_DEVICE, "cannot select the device");
  psl_stats S{};
  psl_status e = run_engine(p, &S);
  if (e != PSL_OK) return e;
  *res = p->result;
  if (stats) *stats = S;
  return PSL_OK;
}

// view of LP k's reduced problem (K = 1: the whole reduced problem)
static psl_reduced_view reduced_view(const psl_presolver* p, int k) {
  const LpRed& b = p->h_lpr[k];
  const LpRed& e = p->h_lpr[k + 1];
  psl_reduced_view v;
  v.m = e.rb - b.rb;
  v.n = e.cb - b.cb;
  v.nnz = e.eb - b.eb;
  v.row_ptr = p->red.row_ptr + b.rb + k;
  v.col_idx = p->red.col_idx + b.eb;
  v.val = p->red.val + b.eb;
  v.col_ptr = p->red.col_ptr + b.cb + k;
  v.row_idx = p->red.row_idx + b.qb;
  v.cval = p->red.cval + b.qb;
  v.lhs = p->red.lhs + b.rb;
  v.rhs = p->red.rhs + b.rb;
  v.lb = p->red.lb + b.cb;
  v.ub = p->red.ub + b.cb;
  v.c = p->red.c + b.cb;
  v.obj_offset = p->K > 1 ? p->h_off[k] : p->red_off;
  v.row_map = p->red.row_map + b.rb;
  v.col_map = p->red.col_map + b.cb;
  v.row_class = p->red.row_class + b.rb;
  v.col_class = p->red.col_class + b.cb;
  return v;
}

static bool has_reduced(const psl_presolver* p, int k) {
  return p->state == 1 && k >= 0 && k < (int)p->lp_result.size() &&
         (p->lp_result[k] == PSL_RES_REDUCED || p->lp_result[k] == PSL_RES_UNCHANGED);
}

extern "C" psl_status psl_reduced_problem(const psl_presolver* p, psl_reduced_view* out) {
  if (!p || !out) return PSL_ERR_INVALID;
  if (!has_reduced(p, 0)) {
    const_cast<psl_presolver*>(p)->err = "no reduced problem: run first (and the result must not be infeasible)";
    return PSL_ERR_STATE;
  }
  *out = reduced_view(p, 0);
  return PSL_OK;
}

// records of LP k on the host (K = 1: all records)
static psl_status fetch_lp_records(psl_presolver* p, int k, const std::vector<psl_record>** out) {
  if (p->K == 1) {
    if (!p->host_rec_valid) {
      // the flushed records, then the device stack's
      int64_t dev = p->rec_count - p->rec_flushed;
      p->host_rec.resize((size_t)p->rec_count);
      if (p->rec_flushed) std::memcpy(p->host_rec.data(), p->flushed.data(), p->rec_flushed * sizeof(psl_record));
      if (dev) {
        HIPCHK(p, hipMemcpyAsync(p->host_rec.data() + p->rec_flushed, p->rec, dev * sizeof(Record),
                                 hipMemcpyDeviceToHost, p->stream));
        HIPCHK(p, hipStreamSynchronize(p->stream));
      }
      p->host_rec_valid = true;
    }
    *out = &p->host_rec;
    return PSL_OK;
  }
  if (p->lp_host_rec.size() != (size_t)p->K) {
    p->lp_host_rec.assign(p->K, {});
    p->lp_rec_valid.assign(p->K, 0);
  }
  if (!p->lp_rec_valid[k]) {
    int64_t a = p->h_rec_off[k], c = p->h_rec_off[k + 1] - a;
    auto& v = p->lp_host_rec[k];
    v.resize((size_t)c);
    if (c) {
      HIPCHK(p, hipMemcpyAsync(v.data(), p->rec_lp + a, c * sizeof(Record), hipMemcpyDeviceToHost, p->stream));
      HIPCHK(p, hipStreamSynchronize(p->stream));
    }
    p->lp_rec_valid[k] = 1;
  }
  *out = &p->lp_host_rec[k];
  return PSL_OK;
}

static psl_status records_of(psl_presolver* p, int k, int64_t* count, psl_record* out, int64_t cap) {
  if (p->state != 1) return fail(p, PSL_ERR_STATE, "no run yet");
  int64_t c = p->K == 1 ? p->rec_count : p->h_rec_off[k + 1] - p->h_rec_off[k];
  if (out) {
    if (cap < c) return fail(p, PSL_ERR_CAPACITY, "record buffer too small");
    const std::vector<psl_record>* v = nullptr;
    psl_status st = fetch_lp_records(p, k, &v);
    if (st != PSL_OK) return st;
    if (c) std::memcpy(out, v->data(), c * sizeof(psl_record));
  }
  *count = c;
  return PSL_OK;
}

extern "C" psl_status psl_records(const psl_presolver* cp, int64_t* count, psl_record* out, int64_t cap) {
  psl_presolver* p = const_cast<psl_presolver*>(cp);
  if (!p || !count) return PSL_ERR_INVALID;
  return records_of(p, 0, count, out, cap);
}

// LP k's rows of the original LP (columns numbered within the LP), copied to
// the host
static psl_status host_rows(psl_presolver* p, int k, HostRows& A) {
  int64_t r0 = p->K == 1 ? 0 : p->h_row0[k], r1 = p->K == 1 ? p->m : p->h_row0[k + 1];
  int64_t c0 = p->K == 1 ? 0 : p->h_col0[k];
  int64_t m = r1 - r0;
  A.rp.resize(m + 1);
  HIPCHK(p, hipMemcpy(A.rp.data(), p->d.rp + r0, (m + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  int64_t e0 = A.rp[0], e1 = A.rp[m];
  A.ci.resize(e1 - e0);
  A.va.resize(e1 - e0);
  if (e1 > e0) {
    HIPCHK(p, hipMemcpy(A.ci.data(), p->d.ci + e0, (e1 - e0) * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(p, hipMemcpy(A.va.data(), p->d.va + e0, (e1 - e0) * sizeof(double), hipMemcpyDeviceToHost));
  }
  for (auto& v : A.rp) v -= (int32_t)e0;
  if (c0)
    for (auto& v : A.ci) v -= (int32_t)c0;
  return PSL_OK;
}

psl_status psl::engine_host_rows(psl_presolver* p, int k, HostRows& A) { return host_rows(p, k, A); }

// LP k's columns of the original (canonicalised) LP and their costs, copied
// to the host; rows numbered within the LP
static psl_status host_cols(psl_presolver* p, int k, HostCols& A) {
  int64_t c0 = p->K == 1 ? 0 : p->h_col0[k], c1 = p->K == 1 ? p->n : p->h_col0[k + 1];
  int64_t r0 = p->K == 1 ? 0 : p->h_row0[k];
  int64_t n = c1 - c0;
  A.cp.resize(n + 1);
  A.c.resize(n);
  // substitutions rewrite the rows: the dual postsolve reads the input's columns
  const int32_t* dcp = p->cp0 ? p->cp0 : p->d.cp;
  const int32_t* dri = p->ri0 ? p->ri0 : p->d.ri;
  const double* dcva = p->cva0 ? p->cva0 : p->d.cva;
  HIPCHK(p, hipMemcpy(A.cp.data(), dcp + c0, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (n) HIPCHK(p, hipMemcpy(A.c.data(), p->c_mut + c0, n * sizeof(double), hipMemcpyDeviceToHost));
  int64_t q0 = A.cp[0], q1 = A.cp[n];
  A.ri.resize(q1 - q0);
  A.cva.resize(q1 - q0);
  if (q1 > q0) {
    HIPCHK(p, hipMemcpy(A.ri.data(), dri + q0, (q1 - q0) * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(p, hipMemcpy(A.cva.data(), dcva + q0, (q1 - q0) * sizeof(double), hipMemcpyDeviceToHost));
  }
  for (auto& v : A.cp) v -= (int32_t)q0;
  if (r0)
    for (auto& v : A.ri) v -= (int32_t)r0;
  return PSL_OK;
}

// postsolve of LP k: the primal solution, and with y_red the row duals and
// reduced costs as well
static psl_status postsolve_of(psl_presolver* p, int k, const double* x_red, const double* y_red,
                               const double* z_red, double* x, double* y, double* z) {
  (void)z_red;  // reduced costs are recomputed from the row duals
  if (!has_reduced(p, k)) return fail(p, PSL_ERR_STATE, "no reduced problem to postsolve");
  psl_reduced_view v = reduced_view(p, k);
  int32_t n = p->K == 1 ? p->n : p->h_col0[k + 1] - p->h_col0[k];
  int32_t m = p->K == 1 ? p->m : p->h_row0[k + 1] - p->h_row0[k];
  if ((n > 0 && !x) || (v.n > 0 && !x_red)) return fail(p, PSL_ERR_INVALID, "null solution array");
  if (y_red && ((m > 0 && !y) || (n > 0 && !z) || (v.m > 0 && !y_red)))
    return fail(p, PSL_ERR_INVALID, "null dual array");
  const std::vector<psl_record>* rec = nullptr;
  psl_status st = fetch_lp_records(p, k, &rec);
  if (st != PSL_OK) return st;
  std::string err;
  HostRows R;
  bool need_rows = records_need_rows(rec->data(), (int64_t)rec->size());
  if (need_rows) {
    st = host_rows(p, k, R);
    if (st != PSL_OK) return st;
  }
  st = postsolve_primal(rec->data(), (int64_t)rec->size(), v.col_map, n, v.n, x_red, x, need_rows ? &R : nullptr,
                        p->s.inf_value, &err);
  if (st != PSL_OK) {
    p->err = err;
    return st;
  }
  if (!y_red) return PSL_OK;
  std::vector<int32_t> rmap(v.m);
  if (v.m) HIPCHK(p, hipMemcpy(rmap.data(), v.row_map, v.m * sizeof(int32_t), hipMemcpyDeviceToHost));
  HostCols A;
  st = host_cols(p, k, A);
  if (st != PSL_OK) return st;
  postsolve_dual(rec->data(), (int64_t)rec->size(), m, n, rmap, y_red, A, y, z);
  return PSL_OK;
}

psl_status psl::engine_host_cols(psl_presolver* p, int k, HostCols& A) { return host_cols(p, k, A); }

extern "C" psl_status psl_postsolve(psl_presolver* p, const double* x_red, const double* y_red, const double* z_red,
                                    double* x, double* y, double* z) {
  if (!p) return PSL_ERR_INVALID;
  return postsolve_of(p, 0, x_red, y_red, z_red, x, y, z);
}

extern "C" void psl_presolve_free(psl_presolver* p) {
  if (!p) return;
  (void)hipSetDevice(p->s.device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  for (void* a : p->allocs) (void)hipFree(a);
  for (void* a : p->hallocs) (void)hipHostFree(a);
  if (!p->borrowed_events)
    for (auto& e : p->ev)
      if (e) (void)hipEventDestroy(e);
  delete p;
}

void psl::set_create_error(const std::string& msg) { g_create_error = msg; }

extern "C" const char* psl_last_error(const psl_presolver* p) {
  if (!p) return g_create_error.c_str();
  return p->err.c_str();
}

// ---------------------------------------------------------------------------
// batched presolve
// ---------------------------------------------------------------------------
// One presolve of lp with every device array carved from dev_scratch and the
// host staging from host_stage (see psl_presolve_noalloc): create, run and a
// copy of the reduced problem and the records into the caller's buffers, in
// one call that allocates no device or pinned host memory.
psl_status psl::engine_run_static(const psl_lp* lp, const psl_settings* s, unsigned char* dev_scratch,
                                  size_t dev_bytes, unsigned char* host_stage, size_t host_bytes, hipEvent_t* ev,
                                  psl_noalloc_out* out, psl_result* res, psl_stats* stats, std::string* err) {
  std::unique_ptr<psl_presolver> h(new psl_presolver());
  psl_presolver* p = h.get();
  take_settings(p, s);
  p->carve = dev_scratch;
  p->carve_cap = dev_bytes;
  p->hcarve = host_stage;
  p->hcarve_cap = host_bytes;
  p->borrowed_events = true;
  for (int k = 0; k < 8; ++k) p->ev[k] = ev[k];
  p->cap_m = lp->m;
  p->cap_n = lp->n;
  p->cap_nnz = lp->nnz;
  p->cap_K = 1;
  set_sizes(p, 1, lp->m, lp->n, lp->nnz);
  psl_status st = setup_arena(p);
  // the scratch keeps the previous call's contents, laid out for another
  // LP: clear the part this LP uses, so it starts as fresh memory would
  if (st == PSL_OK) fill_i32((int32_t*)dev_scratch, 0, (int64_t)(p->carve_used / 4), p->stream);
  if (st == PSL_OK) st = ingest(p, lp);
  psl_stats S{};
  if (st == PSL_OK) st = run_engine(p, &S);
  if (st == PSL_OK && p->rec_count > out->records_cap)
    st = fail(p, PSL_ERR_CAPACITY, "records_cap (" + std::to_string(out->records_cap) + ") below the " +
                                       std::to_string(p->rec_count) + " records of this presolve");
  if (st == PSL_OK && has_reduced(p, 0)) {
    psl_reduced_view v = reduced_view(p, 0);
    hipStream_t q = p->stream;
    auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
      return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, q) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    auto chain = [&](hipError_t x) {
      if (e == hipSuccess) e = x;
    };
    chain(cp(out->row_ptr, v.row_ptr, (v.m + 1) * sizeof(int32_t)));
    chain(cp(out->col_idx, v.col_idx, v.nnz * sizeof(int32_t)));
    chain(cp(out->val, v.val, v.nnz * sizeof(double)));
    chain(cp(out->col_ptr, v.col_ptr, (v.n + 1) * sizeof(int32_t)));
    chain(cp(out->row_idx, v.row_idx, v.nnz * sizeof(int32_t)));
    chain(cp(out->cval, v.cval, v.nnz * sizeof(double)));
    chain(cp(out->lhs, v.lhs, v.m * sizeof(double)));
    chain(cp(out->rhs, v.rhs, v.m * sizeof(double)));
    chain(cp(out->lb, v.lb, v.n * sizeof(double)));
    chain(cp(out->ub, v.ub, v.n * sizeof(double)));
    chain(cp(out->c, v.c, v.n * sizeof(double)));
    chain(cp(out->row_map, v.row_map, v.m * sizeof(int32_t)));
    chain(cp(out->col_map, v.col_map, v.n * sizeof(int32_t)));
    chain(cp(out->row_class, v.row_class, v.m));
    chain(cp(out->col_class, v.col_class, v.n));
    out->m_out = v.m;
    out->n_out = v.n;
    out->nnz_out = v.nnz;
    out->obj_offset = v.obj_offset;
    if (e != hipSuccess) st = fail(p, PSL_ERR_DEVICE, std::string("HIP error copying the reduced problem: ") +
                                                          hipGetErrorString(e));
  } else if (st == PSL_OK) {
    out->m_out = out->n_out = 0;
    out->nnz_out = 0;
    out->obj_offset = 0.0;
  }
  if (st == PSL_OK && p->rec_count &&
      hipMemcpyAsync(out->records, p->rec, p->rec_count * sizeof(Record), hipMemcpyDeviceToDevice, p->stream) !=
          hipSuccess)
    st = fail(p, PSL_ERR_DEVICE, "HIP error copying the records");
  if (st == PSL_OK && hipStreamSynchronize(p->stream) != hipSuccess) st = fail(p, PSL_ERR_DEVICE, "HIP error");
  if (st == PSL_OK) {
    out->records_out = p->rec_count;
    *res = p->result;
    if (stats) *stats = S;
  } else {
    *err = p->err;
    (void)hipStreamSynchronize(p->stream);
  }
  return st;
}

struct psl_batch {
  psl_presolver* p = nullptr;
};

namespace {
thread_local std::string g_batch_error = "no error";
}

std::string psl::check_batch(int32_t k, const psl_lp* lps, int64_t& M, int64_t& Nc, int64_t& Z) {
  M = Nc = Z = 0;
  if (k < 1) return "a batch needs k >= 1 LPs";
  for (int32_t t = 0; t < k; ++t) {
    std::string e = check_lp_shape(&lps[t]);
    if (!e.empty()) return "LP " + std::to_string(t) + ": " + e;
    if (lps[t].mem != lps[0].mem) return "all LPs of a batch must have the same mem kind";
    M += lps[t].m;
    Nc += lps[t].n;
    Z += lps[t].nnz;
  }
  if (Z >= ((int64_t)1 << 30)) return "total nnz of a batch must be below 2^30";
  if (M >= ((int64_t)1 << 30) || Nc >= ((int64_t)1 << 30)) return "a batch must have below 2^30 rows and columns";
  return "";
}

static psl_status batch_load(psl_presolver* p, int32_t k, const psl_lp* lps) {
  p->err_lp = -1;
  if (k == 1) {
    set_sizes(p, 1, lps[0].m, lps[0].n, lps[0].nnz);
    return ingest(p, &lps[0]);
  }
  return ingest_batch(p, k, lps);
}

extern "C" psl_status psl_batch_create(int32_t k, const psl_lp* lps, const psl_settings* s, psl_batch** out) {
  if (!lps || !out) {
    g_batch_error = "null argument";
    return PSL_ERR_INVALID;
  }
  psl_settings def;
  psl_settings_default(&def);
  if (!s) s = &def;
  int64_t M, Nc, Z;
  std::string e = check_settings(s);
  if (e.empty()) e = check_batch(k, lps, M, Nc, Z);
  if (!e.empty()) {
    g_batch_error = e;
    return PSL_ERR_INVALID;
  }
  if (s->device_records > 0) {
    g_batch_error = "device_records (a flushed record stack) is for single-LP presolvers";
    return PSL_ERR_UNSUPPORTED;
  }
  if (hipSetDevice(s->device) != hipSuccess) {
    g_batch_error = "cannot select the device";
    return PSL_ERR_DEVICE;
  }
  psl_presolver* p = new psl_presolver();
  p->s = *s;
  p->s.bin_thresholds = nullptr;
  if (s->bin_thresholds) {
    p->thresholds[0] = s->bin_thresholds[0];
    p->thresholds[1] = s->bin_thresholds[1];
    if (s->n_bins == 3) p->thresholds[2] = s->bin_thresholds[2];
  }
  p->stream = (hipStream_t)s->stream;
  p->sweep_mode = s->split_sweep ? 2 : MODE_ROUND;
  if (const char* e = std::getenv("PSL_TRACE")) p->trace = std::atoi(e) != 0;
  p->cap_m = (int32_t)M;
  p->cap_n = (int32_t)Nc;
  p->cap_nnz = Z;
  p->cap_K = k;
  psl_status st = setup_arena(p);
  if (st == PSL_OK) st = batch_load(p, k, lps);
  if (st != PSL_OK) {
    g_batch_error = p->err;
    psl_presolve_free(p);
    return st;
  }
  psl_batch* b = new psl_batch();
  b->p = p;
  *out = b;
  return PSL_OK;
}

extern "C" psl_status psl_batch_reload(psl_batch* b, int32_t k, const psl_lp* lps) {
  if (!b || !lps) return PSL_ERR_INVALID;
  psl_presolver* p = b->p;
  int64_t M, Nc, Z;
  std::string e = check_batch(k, lps, M, Nc, Z);
  if (!e.empty()) return fail(p, PSL_ERR_INVALID, e);
  if (k > p->cap_K || M > p->cap_m || Nc > p->cap_n || Z > p->cap_nnz)
    return fail(p, PSL_ERR_CAPACITY, "the LPs exceed the batch's capacity");
  if (hipSetDevice(p->s.device) != hipSuccess) return fail(p, PSL_ERR_DEVICE, "cannot select the device");
  psl_status st = batch_load(p, k, lps);
  if (st != PSL_OK) p->state = 2;
  return st;
}

extern "C" psl_status psl_batch_run(psl_batch* b, psl_result* res, psl_stats* total) {
  if (!b || !res) return PSL_ERR_INVALID;
  psl_presolver* p = b->p;
  if (p->state != 0) return fail(p, PSL_ERR_STATE, "run needs a fresh create or reload");
  if (hipSetDevice(p->s.device) != hipSuccess) return fail(p, PSL_ERR_DEVICE, "cannot select the device");
  psl_stats S{};
  psl_status e = run_engine(p, &S);
  if (e != PSL_OK) return e;
  for (int k = 0; k < p->K; ++k) res[k] = p->lp_result[k];
  if (total) *total = S;
  return PSL_OK;
}

static bool batch_idx_ok(const psl_batch* b, int32_t idx) {
  return b && idx >= 0 && idx < b->p->K;
}

void psl::engine_lp_stats(const psl_presolver* p, int idx, psl_stats* out) {
  psl_stats S = p->stats;
  const LpState& L = p->lst[idx];
  S.rounds = L.rounds;
  S.outer_cycles = std::max(1, L.cycles);
  S.records = p->K == 1 ? p->rec_count : p->h_rec_off[idx + 1] - p->h_rec_off[idx];
  S.nnz_in = p->K == 1 ? p->nnz : p->h_z0[idx + 1] - p->h_z0[idx];
  if (has_reduced(p, idx)) {
    psl_reduced_view v = reduced_view(p, idx);
    S.nnz_out = v.nnz;
    S.m_out = v.m;
    S.n_out = v.n;
  } else {
    S.nnz_out = 0;
    S.m_out = S.n_out = 0;
  }
  *out = S;
}

extern "C" psl_status psl_batch_stats(const psl_batch* b, int32_t idx, psl_stats* out) {
  if (!batch_idx_ok(b, idx) || !out) return PSL_ERR_INVALID;
  if (b->p->state != 1) return fail(b->p, PSL_ERR_STATE, "no run yet");
  engine_lp_stats(b->p, idx, out);
  return PSL_OK;
}

extern "C" psl_status psl_batch_reduced_problem(const psl_batch* b, int32_t idx, psl_reduced_view* out) {
  if (!batch_idx_ok(b, idx) || !out) return PSL_ERR_INVALID;
  if (!has_reduced(b->p, idx))
    return fail(b->p, PSL_ERR_STATE, "no reduced problem: run first (and the result must not be infeasible)");
  *out = reduced_view(b->p, idx);
  return PSL_OK;
}

extern "C" psl_status psl_batch_records(const psl_batch* b, int32_t idx, int64_t* count, psl_record* out,
                                        int64_t cap) {
  if (!batch_idx_ok(b, idx) || !count) return PSL_ERR_INVALID;
  return records_of(b->p, idx, count, out, cap);
}

extern "C" psl_status psl_batch_postsolve(psl_batch* b, int32_t idx, const double* x_red, const double* y_red,
                                          const double* z_red, double* x, double* y, double* z) {
  if (!batch_idx_ok(b, idx)) return PSL_ERR_INVALID;
  return postsolve_of(b->p, idx, x_red, y_red, z_red, x, y, z);
}

extern "C" void psl_batch_free(psl_batch* b) {
  if (!b) return;
  psl_presolve_free(b->p);
  delete b;
}

extern "C" const char* psl_batch_last_error(const psl_batch* b) {
  if (!b) return g_batch_error.c_str();
  return b->p->err.c_str();
}

// ---------------------------------------------------------------------------
// engine interface for the server
// ---------------------------------------------------------------------------
psl_presolver* psl::engine_new(const psl_settings* s, int32_t cap_m, int32_t cap_n, int64_t cap_nnz, int32_t cap_K,
                               psl_status* st, std::string* err) {
  psl_presolver* p = new psl_presolver();
  p->s = *s;
  p->s.bin_thresholds = nullptr;
  if (s->bin_thresholds) {
    p->thresholds[0] = s->bin_thresholds[0];
    p->thresholds[1] = s->bin_thresholds[1];
    if (s->n_bins == 3) p->thresholds[2] = s->bin_thresholds[2];
  }
  p->stream = (hipStream_t)s->stream;
  p->sweep_mode = s->split_sweep ? 2 : MODE_ROUND;
  p->cap_m = cap_m;
  p->cap_n = cap_n;
  p->cap_nnz = cap_nnz;
  p->cap_K = cap_K;
  p->state = 2;  // nothing loaded
  *st = setup_arena(p);
  if (*st != PSL_OK) {
    *err = p->err;
    psl_presolve_free(p);
    return nullptr;
  }
  return p;
}

void psl::engine_free(psl_presolver* p) { psl_presolve_free(p); }

psl_status psl::engine_load(psl_presolver* p, int32_t k, const psl_lp* lps) {
  psl_status st = batch_load(p, k, lps);
  if (st != PSL_OK) p->state = 2;
  return st;
}

psl_status psl::engine_run(psl_presolver* p, psl_stats* out) {
  if (p->state != 0) return fail(p, PSL_ERR_STATE, "run needs a fresh load");
  return run_engine(p, out);
}

psl_result psl::engine_result(const psl_presolver* p, int k) { return p->lp_result[k]; }

bool psl::engine_has_reduced(const psl_presolver* p, int k) { return has_reduced(p, k); }

psl_reduced_view psl::engine_view(const psl_presolver* p, int k) { return reduced_view(p, k); }

int64_t psl::engine_records(const psl_presolver* p, int k, const void** dev) {
  if (p->K == 1) {
    *dev = p->rec;
    return p->rec_count;
  }
  *dev = p->rec_lp + p->h_rec_off[k];
  return p->h_rec_off[k + 1] - p->h_rec_off[k];
}

const std::string& psl::engine_error(const psl_presolver* p) { return p->err; }

int32_t psl::engine_error_lp(const psl_presolver* p) { return p->err_lp; }

size_t psl::engine_arena_bytes(const psl_presolver* p) { return p->arena_bytes; }

// ---------------------------------------------------------------------------
// autotuning of the launch shapes
// ---------------------------------------------------------------------------
extern "C" psl_status psl_tune(int32_t k, const psl_lp* lps, const psl_settings* s, int32_t reps, psl_tuning* out) {
  if (!lps || !out || k < 1 || reps < 1) {
    g_batch_error = "psl_tune needs k >= 1 LPs, reps >= 1 and an output";
    return PSL_ERR_INVALID;
  }
  psl_settings base;
  if (s) base = *s;
  else psl_settings_default(&base);
  // the default shape first, then wavefront thresholds, chunk sizes, splits
  const int32_t t0s[] = {512, 256, 128, 64};
  const int32_t t1s[] = {PASS_LEN, 4 * PASS_LEN};
  const int32_t t2s[] = {8, 4};
  psl_tuning best{};
  best.ms_best = -1.0;
  std::vector<psl_result> res(k), ref;
  int64_t ref_records = -1;
  int cand = 0;
  for (int32_t t2 : t2s)
  for (int32_t t1 : t1s)
    for (int32_t t0 : t0s)
      for (int split = 0; split < 2; ++split) {
        psl_settings c = base;
        int32_t thr[3] = {t0, t1, t2};
        c.bin_thresholds = thr;
        c.n_bins = 3;
        c.split_sweep = split;
        psl_batch* b = nullptr;
        psl_status st = psl_batch_create(k, lps, &c, &b);
        if (st != PSL_OK) return st;
        psl_stats S{};
        std::vector<double> ms;
        st = psl_batch_run(b, res.data(), &S);
        for (int r = 0; r < reps && st == PSL_OK; ++r) {
          st = psl_batch_reload(b, k, lps);
          if (st == PSL_OK) st = psl_batch_run(b, res.data(), &S);
          if (st == PSL_OK) ms.push_back(S.ms_total + S.ms_ingest);
        }
        if (st != PSL_OK) {
          g_batch_error = b->p->err;
          psl_batch_free(b);
          return st;
        }
        psl_batch_free(b);
        if (ref_records < 0) {
          ref_records = S.records;
          ref = res;
        } else if (S.records != ref_records || res != ref) {
          g_batch_error = "tuning candidates gave different results";
          return PSL_ERR_DEVICE;
        }
        // the fastest rep: timing noise only ever adds
        double fast = *std::min_element(ms.begin(), ms.end());
        if (cand == 0) best.ms_default = fast;
        if (best.ms_best < 0 || fast < best.ms_best) {
          best.ms_best = fast;
          best.bin_thresholds[0] = t0;
          best.bin_thresholds[1] = t1;
          best.bin_thresholds[2] = t2;
          best.split_sweep = split;
        }
        ++cand;
      }
  best.candidates = cand;
  *out = best;
  return PSL_OK;
}
