// capi.hip -- libpsl's C-ABI: device arena, ingest, the round controller
// (section 3.1: rounds until nothing tightens or a cap is hit; then parallel
// rows, section 3.2; repeated for a few outer cycles), compaction and the
// host postsolve (section 3.3).
//
// Control crosses to the host once per round: a 64-byte flag block (records
// emitted, infeasible / unbounded) is read back to decide whether to go on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/psl.h"
#include "psl_kern.h"
#include "sweep.h"

using namespace psl;

namespace {

thread_local std::string g_create_error = "no error";

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

struct View {
  BinEnt* bins = nullptr;
  LongChunk* chunks = nullptr;
  int32_t off[NBINS + 1] = {0};
  int32_t nchunks = 0;
  int64_t rows = 0, nnz = 0;
};

struct psl_presolver {
  Dev d{};
  psl_settings s{};
  hipStream_t stream = nullptr;
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  std::vector<void*> allocs;
  std::string err = "no error";

  // staging and persistent scratch
  double *lb_in = nullptr, *ub_in = nullptr, *c_mut = nullptr;
  IngestScratch isc{};
  int32_t* ws = nullptr;
  const uint32_t* colid = nullptr;
  int32_t* bin_counts_dev = nullptr;
  int32_t bin_counts[NBINS] = {0};
  int32_t thresholds[2] = {512, PASS_LEN};  // longest wavefront row, chunk positions
  SweepGrid grid{};
  int64_t chunk_cap = 0, long_cap = 0, cand_cap = 0;
  int32_t* cand_cnt = nullptr;
  // bin views: the master lists hold the active rows (filtered after
  // removals); a selection holds the active rows touched by a column change
  // since they were last swept
  BinEnt *bins_a = nullptr, *bins_b = nullptr, *bins_s = nullptr;
  LongChunk *chunks_a = nullptr, *chunks_b = nullptr, *chunks_s = nullptr;
  int32_t* rebin_dev = nullptr;  // [NBINS+1] new offsets, then 3 totals
  View master, cur;

  // records
  Record* rec = nullptr;
  int64_t rec_cap = 0, rec_count = 0;
  std::vector<psl_record> host_rec;
  bool host_rec_valid = false;

  ParScratch par{};
  CompactScratch cmp{};
  Reduced red{};
  int32_t red_m = 0, red_n = 0;
  int64_t red_nnz = 0;
  double red_off = 0.0;
  double obj_offset = 0.0;

  Flags* hflags = nullptr;  // pinned
  int32_t* htot = nullptr;  // pinned [4] + offset
  double* hoff = nullptr;

  int state = 0;  // 0 loaded, 1 ran
  int sweep_mode = MODE_ROUND;  // PSL_SWEEP_SPLIT=1: three launches by register class
  psl_result result = PSL_RES_UNCHANGED;
  psl_stats stats{};
  double ms_ingest = 0.0;
  hipEvent_t ev[8] = {nullptr};
};

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
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
    return PSL_ERR_OOM;
  }
  p->allocs.push_back(ptr);
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
}

static std::string check_settings(const psl_settings* s) {
  if (s->max_rounds < 1 || s->max_outer < 1 || (int64_t)s->max_outer * (s->max_rounds + 1) + 1 > 65535)
    return "invalid round limits";
  if (!(s->feas_tol >= 0) || !(s->fix_tol >= 0) || !(s->min_improve >= 0) || !(s->par_tol >= 0) ||
      !(s->inf_value > 0) || !(s->coef_tol >= 0))
    return "invalid tolerance";
  if (s->bin_thresholds) {
    if (s->n_bins != 2) return "bin_thresholds needs n_bins = 2";
    int a = s->bin_thresholds[0], b = s->bin_thresholds[1];
    if (a < 16 || a > 512) return "bin_thresholds[0] (longest wavefront row) must be in [16, 512]";
    if (b < PASS_LEN || b > PASS_LEN * long_max_passes() || (b & (b - 1)) != 0)
      return "bin_thresholds[1] (chunk positions) must be a power of two >= 2048";
  }
  return "";
}

static std::string check_lp_shape(const psl_lp* lp) {
  if (lp->m < 0 || lp->n < 0 || lp->nnz < 0) return "negative size";
  if (lp->nnz >= ((int64_t)1 << 30)) return "nnz must be below 2^30";
  if (lp->m == 0 && lp->nnz != 0) return "entries without rows";
  if (lp->m > 0 && (!lp->row_ptr || !lp->lhs || !lp->rhs)) return "null row array";
  if (lp->n > 0 && (!lp->lb || !lp->ub || !lp->c)) return "null column array";
  if (lp->nnz > 0 && (!lp->col_idx || !lp->val)) return "null matrix array";
  if (lp->mem != PSL_MEM_HOST && lp->mem != PSL_MEM_DEVICE) return "bad mem kind";
  if (!std::isfinite(lp->obj_offset)) return "offset not finite";
  return "";
}

static psl_status setup_arena(psl_presolver* p) {
  int64_t m = p->m, n = p->n, N = p->nnz;
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
  ALLOC(p->bins_b, m);
  ALLOC(p->bins_s, m);
  ALLOC(p->rebin_dev, 16);
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
  wsn = std::max<size_t>(wsn, scan_ws_ints(m + n + 1)) + 64;
  ALLOC(p->ws, wsn);
  p->isc.ws = p->ws;

  // long rows are longer than the wavefront threshold; chunks of >= 2048
  p->long_cap = N / ((int64_t)p->thresholds[0] + 1) + 1;
  p->chunk_cap = N / PASS_LEN + p->long_cap + 1;
  ALLOC(p->chunks_a, p->chunk_cap);
  ALLOC(p->chunks_b, p->chunk_cap);
  ALLOC(p->chunks_s, p->chunk_cap);
  uint8_t* dirty;
  ALLOC(dirty, m);
  LongPart* lpart;
  LongRow* lrow;
  ALLOC(lpart, p->chunk_cap);
  ALLOC(lrow, p->long_cap);

  p->rec_cap = 2 * m + 4 * n + 1024;
  ALLOC(p->rec, p->rec_cap);

  // parallel rows
  int64_t cap = 64;
  while (cap < 2 * m) cap <<= 1;
  p->par.cap = cap;
  ALLOC(p->par.table, cap);
  ALLOC(p->par.slot, m);
  ALLOC(p->par.lead, m);
  ALLOC(p->par.side_key, 2 * m);
  ALLOC(p->par.side_src, 2 * m);
  ALLOC(p->par.is_leader, m);
  ALLOC(p->par.vlist, m);
  ALLOC(p->par.hacc, 3 * p->long_cap);

  // compaction
  ALLOC(p->cmp.row_new, m + 1);
  ALLOC(p->cmp.col_new, n + 1);
  ALLOC(p->cmp.terms, n);
  ALLOC(p->cmp.pws, pairwise_ws_doubles(n) + 2);
  ALLOC(p->cmp.totals, 4);
  ALLOC(p->cmp.offset, 1);
  p->cmp.ws = p->ws;
  p->cmp.eflag = p->isc.v0;
  p->cmp.qflag = p->isc.v1;
  p->cmp.rowid1 = p->isc.rowid1;

  Reduced& r = p->red;
  ALLOC(r.row_ptr, m + 1);
  ALLOC(r.col_idx, N);
  ALLOC(r.val, N);
  ALLOC(r.col_ptr, n + 1);
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

  HIPCHK(p, hipHostMalloc((void**)&p->hflags, sizeof(Flags), hipHostMallocDefault));
  HIPCHK(p, hipHostMalloc((void**)&p->htot, 64 * sizeof(int32_t), hipHostMallocDefault));
  HIPCHK(p, hipHostMalloc((void**)&p->hoff, sizeof(double), hipHostMallocDefault));
  for (auto& e : p->ev) HIPCHK(p, hipEventCreate(&e));

  d.m = (int32_t)m;
  d.n = (int32_t)n;
  d.nnz = N;
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
  d.c = p->c_mut;
  d.col_len = col_len;
  d.row_on = row_on;
  d.row_code = row_code;
  d.col_code = col_code;
  d.row_out = row_out;
  d.cand = cand;
  d.cand_cnt = p->cand_cnt;
  d.flags = flags;
  d.cnt = cnt;
  d.off = off;
  d.rec = p->rec;
  d.bins = p->bins_a;
  d.lchunk = p->chunks_a;
  d.dirty = dirty;
  d.lpart = lpart;
  d.lrow = lrow;
  d.nlong = 0;
  d.nchunks = 0;
  const psl_settings& s = p->s;
  d.cfg = Cfg{s.feas_tol, s.fix_tol, s.min_improve, s.par_tol, s.inf_value, s.coef_tol};
  // every device array the kernels index must exist (allocations are >= 64 B
  // even for empty problems); colid is set once the transposed copy exists
  const void* ptrs[] = {d.rp, d.ci, d.va, d.cp, d.ri, d.cva, d.lhs, d.rhs, d.bnd, d.bkey, d.src, d.c,
                        d.col_len, d.row_on, d.row_code, d.col_code, d.dirty, d.row_out, d.cand, d.cand_cnt,
                        d.flags, d.cnt, d.off, d.rec, d.bins, d.lchunk, d.lpart, d.lrow};
  for (const void* q : ptrs)
    if (!q) return fail(p, PSL_ERR_DEVICE, "internal: a device array was not set up");
  return PSL_OK;
}

static psl_status read_flags(psl_presolver* p) {
  HIPCHK(p, hipMemcpyAsync(p->hflags, p->d.flags, sizeof(Flags), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return PSL_OK;
}

// flags plus the number of row records of the last scan (rows removed)
static psl_status read_round(psl_presolver* p, int64_t rows_total, int32_t* rows_removed) {
  HIPCHK(p, hipMemcpyAsync(p->hflags, p->d.flags, sizeof(Flags), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipMemcpyAsync(p->htot + 32, p->d.off + rows_total, sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  *rows_removed = p->htot[32];
  return PSL_OK;
}

// workgroups per bin from the current bin offsets and chunk count
static void set_grid(psl_presolver* p) {
  const Dev& d = p->d;
  auto cnt = [&](int b) { return d.bin_off[b + 1] - d.bin_off[b]; };
  p->grid.nb[BIN_G4] = (cnt(BIN_G4) + 63) / 64;
  p->grid.nb[BIN_G16] = (cnt(BIN_G16) + 15) / 16;
  p->grid.nb[BIN_W1] = (cnt(BIN_W1) + 3) / 4;
  p->grid.nb[BIN_W4] = (cnt(BIN_W4) + 3) / 4;
  p->grid.nb[BIN_W8] = (cnt(BIN_W8) + 3) / 4;
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

// dst = the active rows of src (only the dirty ones when dirty is set)
static psl_status filter_view(psl_presolver* p, const View& src, BinEnt* bout, LongChunk* cout, bool dirty,
                              View& dst) {
  Dev& d = p->d;
  // scratch: cnt / off (free after the round's emission) and v0 (free between
  // ingest and compaction; k0 / k1 hold the transposed copy's column ids)
  rebin(d, src.bins, src.off, src.chunks, src.nchunks, bout, cout, dirty ? d.dirty : nullptr, d.cnt, d.off,
        p->isc.v0, p->rebin_dev, p->rebin_dev + NBINS + 1, p->ws, p->stream);
  HIPCHK(p, hipMemcpyAsync(p->htot, p->rebin_dev, (NBINS + 4) * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  View v;
  v.bins = bout;
  v.chunks = cout;
  for (int b = 0; b <= NBINS; ++b) v.off[b] = p->htot[b];
  v.rows = p->htot[NBINS + 1];
  v.nnz = p->htot[NBINS + 2];
  v.nchunks = p->htot[NBINS + 3];
  dst = v;
  return PSL_OK;
}

static std::string error_message(int32_t bits, int64_t pos) {
  std::string what;
  if (bits & 1) what = "row_ptr must start at 0, be non-decreasing and end at nnz";
  else if (bits & 2) what = "column index out of range or not strictly ascending within its row";
  else if (bits & 4) what = "coefficient zero or not finite";
  else if (bits & 8) what = "side NaN or infinite on the wrong end";
  else if (bits & 16) what = "bound NaN or infinite on the wrong end";
  else what = "cost not finite";
  return "invalid input: " + what + " (first at index " + std::to_string(pos) + ")";
}

// copy + validate + transpose + bins; the LP's shape equals the handle's
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

  launch_init_state(d, st);  // clears the flag block
  launch_check_rows(d, st);
  check_cols(d, p->lb_in, p->ub_in, p->c_mut, st);
  psl_status s0 = read_flags(p);
  if (s0 != PSL_OK) return s0;
  if (p->hflags->error) return fail(p, PSL_ERR_INVALID, error_message(p->hflags->error, p->hflags->error_pos));

  build_rowid(d, p->isc, st);
  launch_check_entries(d, p->isc.rowid1, st);
  s0 = read_flags(p);
  if (s0 != PSL_OK) return s0;
  if (p->hflags->error) return fail(p, PSL_ERR_INVALID, error_message(p->hflags->error, p->hflags->error_pos));

  // bins (before the transpose: both use k0/k1)
  d.bins = p->bins_a;
  d.lchunk = p->chunks_a;
  build_bins(d, p->thresholds, p->bins_a, p->bin_counts_dev, p->isc, st);
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
  build_long_chunks(d, p->thresholds[1] / PASS_LEN, p->chunks_a, d.cnt, d.off, p->bin_counts_dev, p->ws, st);
  HIPCHK(p, hipMemcpyAsync(p->htot, p->bin_counts_dev, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  s0 = read_flags(p);
  if (s0 != PSL_OK) return s0;
  if (p->hflags->error & 64) return fail(p, PSL_ERR_CAPACITY, "a row is longer than 2^26 entries");
  if (p->htot[0] > p->chunk_cap) return fail(p, PSL_ERR_CAPACITY, "too many long-row chunks");
  d.nchunks = p->htot[0];
  d.colid = nullptr;
  View mv;
  mv.bins = p->bins_a;
  mv.chunks = p->chunks_a;
  for (int b = 0; b <= NBINS; ++b) mv.off[b] = d.bin_off[b];
  mv.nchunks = d.nchunks;
  mv.rows = m;
  mv.nnz = N;
  p->master = mv;
  use_view(p, mv);
  if (p->grid.long_base + (int64_t)p->htot[1] > p->cand_cap)
    return fail(p, PSL_ERR_CAPACITY, "candidate buffer too small for the row bins");

  p->colid = build_csc(d, (int32_t*)d.cp, (int32_t*)d.ri, (double*)d.cva, d.col_len, p->isc, st);
  p->cmp.colid = p->colid;
  d.colid = p->colid;
  HIPCHK(p, hipEventRecord(p->ev[1], st));
  HIPCHK(p, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(p, hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
  p->ms_ingest = ms;
  p->state = 0;
  p->host_rec_valid = false;
  return PSL_OK;
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
  if (!e.empty()) {
    g_create_error = e;
    return PSL_ERR_INVALID;
  }
  if (hipSetDevice(s->device) != hipSuccess) {
    g_create_error = "cannot select the device";
    return PSL_ERR_DEVICE;
  }
  psl_presolver* p = new psl_presolver();
  p->s = *s;
  p->s.bin_thresholds = nullptr;
  if (s->bin_thresholds) {
    p->thresholds[0] = s->bin_thresholds[0];
    p->thresholds[1] = s->bin_thresholds[1];
  }
  p->stream = (hipStream_t)s->stream;
  if (const char* e = std::getenv("PSL_SWEEP_SPLIT")) p->sweep_mode = std::atoi(e) ? 2 : MODE_ROUND;
  p->m = lp->m;
  p->n = lp->n;
  p->nnz = lp->nnz;
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
  if (lp->m != p->m || lp->n != p->n || lp->nnz != p->nnz)
    return fail(p, PSL_ERR_INVALID, "reload needs the same m, n and nnz");
  if (hipSetDevice(p->s.device) != hipSuccess) return fail(p, PSL_ERR_DEVICE, "cannot select the device");
  psl_status st = ingest(p, lp);
  if (st != PSL_OK) p->state = 2;  // unusable until a successful reload
  return st;
}

static psl_status ensure_capacity(psl_presolver* p, int64_t need) {
  if (p->rec_count + need <= p->rec_cap) return PSL_OK;
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

extern "C" psl_status psl_presolve_run(psl_presolver* p, psl_result* res, psl_stats* stats) {
  if (!p || !res) return PSL_ERR_INVALID;
  if (p->state != 0) return fail(p, PSL_ERR_STATE, "run needs a fresh create or reload");
  if (hipSetDevice(p->s.device) != hipSuccess) return fail(p, PSL_ERR_DEVICE, "cannot select the device");
  Dev& d = p->d;
  hipStream_t st = p->stream;
  const psl_settings& s = p->s;
  int64_t m = p->m, n = p->n;
  psl_stats S{};
  S.nnz_in = p->nnz;
  p->rec_count = 0;
  p->host_rec_valid = false;
  p->state = 1;
  HIPCHK(p, hipEventRecord(p->ev[2], st));

  // round 0: input fixings
  launch_init_state(d, st);
  launch_round0_count(d, st);
  scan_excl(d.cnt, d.off, m + n, &d.flags->round_total, p->ws, st);
  launch_round0_emit(d, 0, st);
  psl_status e = read_flags(p);
  if (e != PSL_OK) return e;
  p->rec_count += p->hflags->round_total;
  int round = 0;
  bool infeasible = p->hflags->infeasible != 0, unbounded = false;
  double sweep_ms = 0.0, decide_ms = 0.0, par_ms = 0.0, long_ms = 0.0;

  bool stop = infeasible;
  bool was_incremental = false;
  use_view(p, p->master);
  int outer = 0;
  for (; outer < s.max_outer && !stop; ++outer) {
    for (int r = 0; r < s.max_rounds; ++r) {
      ++round;
      e = ensure_capacity(p, m + 3 * n + 16);
      if (e != PSL_OK) return e;
      HIPCHK(p, hipEventRecord(p->ev[4], st));
      launch_long_stats(d, MODE_ROUND, st);
      HIPCHK(p, hipEventRecord(p->ev[7], st));
      launch_sweep(d, p->grid, p->sweep_mode, st);
      HIPCHK(p, hipEventRecord(p->ev[5], st));
      launch_src(d, p->grid, st);
      launch_count(d, st);
      scan_excl(d.cnt, d.off, m + n, &d.flags->round_total, p->ws, st);
      launch_emit(d, p->rec_count, round, st);
      HIPCHK(p, hipEventRecord(p->ev[6], st));
      int32_t removed = 0;
      e = read_round(p, m, &removed);
      if (e != PSL_OK) return e;
      long_ms += elapsed(p, 4, 7);
      sweep_ms += elapsed(p, 7, 5);
      decide_ms += elapsed(p, 5, 6);
      S.sweep_launches += 1;
      S.sweep_bytes += 12.0 * p->cur.nnz + 24.0 * p->cur.rows + 16.0 * n;
      p->rec_count += p->hflags->round_total;
      if (p->hflags->infeasible) infeasible = true;
      if (p->hflags->unbounded) unbounded = true;
      if (infeasible || unbounded) {
        stop = true;
        break;
      }
      if (p->hflags->round_total == 0) break;
      // keep the master lists on live rows once a sixteenth of them went
      if (removed > 0 && (int64_t)removed * 16 >= p->master.rows) {
        View nv;
        BinEnt* bo = p->master.bins == p->bins_a ? p->bins_b : p->bins_a;
        LongChunk* co = p->master.chunks == p->chunks_a ? p->chunks_b : p->chunks_a;
        e = filter_view(p, p->master, bo, co, false, nv);
        if (e != PSL_OK) return e;
        p->master = nv;
      }
      // Next round: rows none of whose columns changed since they were last
      // swept give the same statistics and no qualifying candidate, so after
      // a round with few column changes only the touched rows are swept.
      int64_t changed_cols = (int64_t)p->hflags->round_total - removed;
      bool incremental = r + 1 < s.max_rounds && changed_cols * 8 < (int64_t)n;
      if (incremental) {
        if (!d.dirty || !d.colid) return fail(p, PSL_ERR_DEVICE, "internal: incremental state not set up");
        mark_dirty(d, !was_incremental, st);
        View sel;
        e = filter_view(p, p->master, p->bins_s, p->chunks_s, true, sel);
        if (e != PSL_OK) return e;
        use_view(p, sel);
      } else {
        use_view(p, p->master);
      }
      was_incremental = incremental;
    }
    use_view(p, p->master);
    was_incremental = false;
    if (stop || !s.enable_parallel_rows) break;
    ++round;
    e = ensure_capacity(p, m + 16);
    if (e != PSL_OK) return e;
    HIPCHK(p, hipEventRecord(p->ev[4], st));
    launch_par_reset(d, p->par, st);
    launch_par_hash(d, p->par, p->grid, st);
    launch_par_verify(d, p->par, st);
    launch_par_count(d, p->par, st);
    scan_excl(d.cnt, d.off, m, &d.flags->round_total, p->ws, st);
    launch_par_emit(d, p->par, p->rec_count, round, st);
    launch_par_drop(d, p->par, st);
    HIPCHK(p, hipEventRecord(p->ev[5], st));
    e = read_flags(p);
    if (e != PSL_OK) return e;
    par_ms += elapsed(p, 4, 5);
    p->rec_count += p->hflags->round_total;
    if (p->hflags->infeasible) {
      infeasible = true;
      stop = true;
      break;
    }
    if (!p->hflags->merged) break;
  }
  if (outer == s.max_outer) outer = s.max_outer;  // cap reached

  psl_result result;
  if (infeasible) result = PSL_RES_INFEASIBLE;
  else if (unbounded) result = PSL_RES_UNBOUNDED_OR_INFEASIBLE;
  else result = p->rec_count ? PSL_RES_REDUCED : PSL_RES_UNCHANGED;

  double cmp_ms = 0.0;
  if (result == PSL_RES_REDUCED || result == PSL_RES_UNCHANGED) {
    use_view(p, p->master);
    HIPCHK(p, hipEventRecord(p->ev[4], st));
    launch_long_stats(d, MODE_COMPACT, st);
    launch_sweep(d, p->grid, MODE_COMPACT, st);
    compact_flags(d, p->cmp, st);
    compact_write(d, p->cmp, p->red, p->obj_offset, st);
    HIPCHK(p, hipEventRecord(p->ev[5], st));
    HIPCHK(p, hipMemcpyAsync(p->htot, p->cmp.totals, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipMemcpyAsync(p->hoff, p->cmp.offset, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    cmp_ms = elapsed(p, 4, 5);
    p->red_m = p->htot[0];
    p->red_n = p->htot[1];
    p->red_nnz = p->htot[2];
    p->red_off = *p->hoff;
    if (p->htot[2] != p->htot[3]) return fail(p, PSL_ERR_DEVICE, "reduced CSR and transposed copy disagree");
  }
  HIPCHK(p, hipEventRecord(p->ev[3], st));
  HIPCHK(p, hipEventSynchronize(p->ev[3]));
  p->result = result;
  S.rounds = round;
  S.outer_cycles = std::min(outer + 1, s.max_outer);
  S.records = p->rec_count;
  S.nnz_out = p->red_nnz;
  S.m_out = p->red_m;
  S.n_out = p->red_n;
  S.ms_ingest = p->ms_ingest;
  S.ms_sweep = sweep_ms;
  S.ms_long = long_ms;
  S.ms_decide = decide_ms;
  S.ms_parallel = par_ms;
  S.ms_compact = cmp_ms;
  S.ms_total = elapsed(p, 2, 3);
  p->stats = S;
  *res = result;
  if (stats) *stats = S;
  return PSL_OK;
}

extern "C" psl_status psl_reduced_problem(const psl_presolver* p, psl_reduced_view* out) {
  if (!p || !out) return PSL_ERR_INVALID;
  if (p->state != 1 || (p->result != PSL_RES_REDUCED && p->result != PSL_RES_UNCHANGED)) {
    const_cast<psl_presolver*>(p)->err = "no reduced problem: run first (and the result must not be infeasible)";
    return PSL_ERR_STATE;
  }
  psl_reduced_view v;
  v.m = p->red_m;
  v.n = p->red_n;
  v.nnz = p->red_nnz;
  v.row_ptr = p->red.row_ptr;
  v.col_idx = p->red.col_idx;
  v.val = p->red.val;
  v.col_ptr = p->red.col_ptr;
  v.row_idx = p->red.row_idx;
  v.cval = p->red.cval;
  v.lhs = p->red.lhs;
  v.rhs = p->red.rhs;
  v.lb = p->red.lb;
  v.ub = p->red.ub;
  v.c = p->red.c;
  v.obj_offset = p->red_off;
  v.row_map = p->red.row_map;
  v.col_map = p->red.col_map;
  v.row_class = p->red.row_class;
  v.col_class = p->red.col_class;
  *out = v;
  return PSL_OK;
}

static psl_status fetch_records(psl_presolver* p) {
  if (p->host_rec_valid) return PSL_OK;
  p->host_rec.resize((size_t)p->rec_count);
  if (p->rec_count) {
    HIPCHK(p, hipMemcpyAsync(p->host_rec.data(), p->rec, p->rec_count * sizeof(Record), hipMemcpyDeviceToHost,
                             p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
  }
  p->host_rec_valid = true;
  return PSL_OK;
}

extern "C" psl_status psl_records(const psl_presolver* cp, int64_t* count, psl_record* out, int64_t cap) {
  psl_presolver* p = const_cast<psl_presolver*>(cp);
  if (!p || !count) return PSL_ERR_INVALID;
  if (p->state != 1) return fail(p, PSL_ERR_STATE, "no run yet");
  if (out) {
    if (cap < p->rec_count) return fail(p, PSL_ERR_CAPACITY, "record buffer too small");
    psl_status st = fetch_records(p);
    if (st != PSL_OK) return st;
    if (p->rec_count) std::memcpy(out, p->host_rec.data(), p->rec_count * sizeof(psl_record));
  }
  *count = p->rec_count;
  return PSL_OK;
}

extern "C" psl_status psl_postsolve(psl_presolver* p, const double* x_red, const double* y_red, const double* z_red,
                                    double* x, double* y, double* z) {
  (void)y;
  (void)z;
  if (!p) return PSL_ERR_INVALID;
  if (y_red || z_red) return fail(p, PSL_ERR_UNSUPPORTED, "dual postsolve is not provided");
  if (p->state != 1 || (p->result != PSL_RES_REDUCED && p->result != PSL_RES_UNCHANGED))
    return fail(p, PSL_ERR_STATE, "no reduced problem to postsolve");
  if ((p->n > 0 && !x) || (p->red_n > 0 && !x_red)) return fail(p, PSL_ERR_INVALID, "null solution array");
  psl_status st = fetch_records(p);
  if (st != PSL_OK) return st;
  std::vector<int32_t> cmap(p->red_n);
  if (p->red_n)
    HIPCHK(p, hipMemcpy(cmap.data(), p->red.col_map, p->red_n * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t j = 0; j < p->n; ++j) x[j] = 0.0;
  for (int32_t k = 0; k < p->red_n; ++k) x[cmap[k]] = x_red[k];
  for (int64_t t = p->rec_count - 1; t >= 0; --t) {
    const psl_record& r = p->host_rec[t];
    if (r.type == REC_FIX_COL || r.type == REC_EMPTY_COL) x[r.j] = r.v[0];
  }
  return PSL_OK;
}

extern "C" void psl_presolve_free(psl_presolver* p) {
  if (!p) return;
  (void)hipSetDevice(p->s.device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  for (void* a : p->allocs) (void)hipFree(a);
  if (p->hflags) (void)hipHostFree(p->hflags);
  if (p->htot) (void)hipHostFree(p->htot);
  if (p->hoff) (void)hipHostFree(p->hoff);
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

extern "C" const char* psl_last_error(const psl_presolver* p) {
  if (!p) return g_create_error.c_str();
  return p->err.c_str();
}
