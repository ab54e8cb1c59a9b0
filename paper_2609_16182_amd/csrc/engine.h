// engine.h -- the presolve engine behind libpsl's C-ABI: the device arena,
// the views of the row bins and the round controller's state, for one LP or a
// batch of LPs. Shared by the presolve / batch entry points and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/psl.h"
#include "psl_kern.h"
#include "sweep.h"

using psl::BinEnt;
using psl::CompactScratch;
using psl::Flags;
using psl::IngestScratch;
using psl::LongChunk;
using psl::LpDesc;
using psl::LpFlags;
using psl::LpOut;
using psl::LpRed;
using psl::LpTab;
using psl::MODE_ROUND;
using psl::NBINS;
using psl::ParScratch;
using psl::Record;
using psl::Reduced;
using psl::SweepGrid;

struct View {
  BinEnt* bins = nullptr;
  LongChunk* chunks = nullptr;
  int32_t off[NBINS + 1] = {0};
  int32_t nchunks = 0;
  int64_t rows = 0, nnz = 0;
};

// host state of one LP of a batch
enum : uint8_t { LP_PROP = 0, LP_WAIT = 1, LP_DONE = 2 };
struct LpState {
  uint8_t phase = LP_PROP;
  bool infeasible = false, unbounded = false;
  int32_t rounds = 0, cycles = 0;
};

// A run is a sequence of units, each one launch (kernels and the
// asynchronous reads of their results, on the engine's stream) and one
// completion (the wait for those reads, then the host's decisions): round 0,
// the propagation rounds of each outer cycle, each cycle's reduction pass, the
// compaction. psl_presolve_run runs them back to back; a stepped server
// interleaves the units of several batches.
enum EngUnit { U_ROUND0 = 0, U_ROUND = 1, U_PASS = 2, U_COMPACT = 3, U_DONE = 4 };
struct EngRun {
  int unit = U_DONE;               // the unit the next launch starts
  int outer = 0, r = 0, round = 0;  // cycle, round in the cycle, rounds so far
  bool consts_current = false;     // row_out current for the compaction
  bool any_feasible = false;       // the compaction unit has work
  double sweep_ms = 0.0, decide_ms = 0.0, par_ms = 0.0, long_ms = 0.0, cmp_ms = 0.0;
  psl_stats S{};
};

struct psl_presolver {
  using Dev = psl::Dev;
  Dev d{};
  psl_settings s{};
  hipStream_t stream = nullptr;
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  // arena capacity (the create-time sizes; a batch reload may use less)
  int32_t cap_m = 0, cap_n = 0, cap_K = 1;
  int64_t cap_nnz = 0;

  // batch (K > 1): device maps and per-LP arrays, pinned host mirrors
  int32_t K = 1;
  int32_t *row_lp = nullptr, *col_lp = nullptr, *lp_row0 = nullptr, *lp_col0 = nullptr, *lp_round = nullptr;
  uint8_t* lp_ok = nullptr;
  LpFlags* lpf = nullptr;
  LpOut* lpo = nullptr;
  LpTab* lpt = nullptr;
  LpRed* lpr = nullptr;
  int64_t* lp_z0 = nullptr;
  LpDesc* descs = nullptr;
  double *lp_off_in = nullptr, *lp_off = nullptr;
  int32_t *h_row0 = nullptr, *h_col0 = nullptr, *h_round = nullptr;
  int64_t* h_z0 = nullptr;
  uint8_t* h_ok = nullptr;
  LpFlags* h_lpf = nullptr;
  LpOut* h_lpo = nullptr;
  LpTab* h_lpt = nullptr;
  LpRed* h_lpr = nullptr;
  LpDesc* h_desc = nullptr;
  double *h_off_in = nullptr, *h_off = nullptr;
  std::vector<LpState> lst;
  std::vector<psl_result> lp_result;
  BinEnt* bins_0 = nullptr;  // the ingest bins of all rows
  LongChunk* chunks_0 = nullptr;
  // records split by LP
  Record* rec_lp = nullptr;
  int64_t split_cap = 0;
  uint32_t *sk0 = nullptr, *sk1 = nullptr;
  int32_t *sv0 = nullptr, *sv1 = nullptr, *sws = nullptr, *rec_off = nullptr;
  std::vector<int32_t> h_rec_off;
  std::vector<std::vector<psl_record>> lp_host_rec;
  std::vector<uint8_t> lp_rec_valid;
  std::vector<void*> allocs, hallocs;
  size_t arena_bytes = 0;   // device bytes allocated by the handle
  std::string err = "no error";
  int32_t err_lp = -1;      // LP of a batch that failed validation, else -1
  int64_t par_slots = 0;

  // staging and persistent scratch
  double *lb_in = nullptr, *ub_in = nullptr, *c_mut = nullptr;
  double* c_work = nullptr;  // the run's costs (c_mut holds the input's)
  IngestScratch isc{};
  int32_t* ws = nullptr;
  const uint32_t* colid = nullptr;
  int32_t* bin_counts_dev = nullptr;
  int32_t bin_counts[NBINS] = {0};
  int32_t thresholds[3] = {512, PASS_LEN, 8};  // longest wavefront row, chunk positions, longest 8-lane row
  SweepGrid grid{};
  int64_t chunk_cap = 0, long_cap = 0, cand_cap = 0;
  int32_t* cand_cnt = nullptr;
  // bin views: a full view holds every active row (of an LP still
  // presolving); a round's selection the rows the device chose for it
  BinEnt *bins_a = nullptr, *bins_s = nullptr;
  LongChunk *chunks_a = nullptr, *chunks_s = nullptr;
  uint8_t* sel_keep = nullptr;   // per-row decisions of the row selection
  int32_t* sel_cnt = nullptr;    // its per-tile counts / offsets
  int32_t* sel_dev = nullptr;    // [NBINS+1] offsets, rows, nonzeros, chunks of a full view
  View cur;

  // records
  Record* rec = nullptr;
  int64_t rec_cap = 0, rec_count = 0;
  // the postsolve stack with flushing (settings.device_records > 0): records
  // [0, rec_flushed) are in `flushed` on the host, the rest on the device
  // from rec[0]; new records go to rec[rec_count - rec_flushed]
  int64_t rec_flushed = 0, flushes = 0;
  std::vector<psl_record> flushed;
  std::vector<psl_record> host_rec;
  bool host_rec_valid = false;

  ParScratch par{};
  psl::ColScratch pc{};  // parallel columns (allocated when enabled)
  psl::DblScratch dbl{};  // doubleton substitution (allocated when enabled)
  psl::DomScratch dom{};  // dominated columns (allocated when enabled)
  // the input's transposed copy, kept when substitutions rewrite the rows (the
  // dual postsolve reads the input's columns)
  int32_t *cp0 = nullptr, *ri0 = nullptr;
  double* cva0 = nullptr;
  CompactScratch cmp{};
  Reduced red{};
  int32_t red_m = 0, red_n = 0;
  int64_t red_nnz = 0;
  double red_off = 0.0;
  double obj_offset = 0.0;

  Flags* hflags = nullptr;  // pinned
  int32_t* htot = nullptr;  // pinned [4] + offset
  double* hoff = nullptr;

  // Static-scratch mode (psl_presolve_noalloc): device arrays are carved from
  // one caller-provided region and host staging from a static buffer; the
  // HIP events are borrowed. Nothing is allocated or freed by the handle.
  unsigned char* carve = nullptr;
  size_t carve_cap = 0, carve_used = 0;
  unsigned char* hcarve = nullptr;
  size_t hcarve_cap = 0, hcarve_used = 0;
  bool borrowed_events = false;

  int state = 0;  // 0 loaded, 1 ran
  int sweep_mode = MODE_ROUND;  // 2: three launches by register class
  bool trace = false;  // PSL_TRACE=1: one line per round on stderr
  // after a round changing fewer than n / incr_factor columns only touched
  // rows are swept; with fewer than n / count_factor bounds made finite the
  // infinite-contribution counts are kept and inert rows skipped
  int incr_factor = 4, count_factor = 16;
  psl_result result = PSL_RES_UNCHANGED;
  psl_stats stats{};
  double ms_ingest = 0.0;
  hipEvent_t ev[8] = {nullptr};
  EngRun run;
};

namespace psl {

std::string check_settings(const psl_settings* s);
std::string check_lp_shape(const psl_lp* lp);
// k LPs of one batch: shapes checked, totals returned
std::string check_batch(int32_t k, const psl_lp* lps, int64_t& M, int64_t& Nc, int64_t& Z);
// an engine with room for LPs of these total sizes (no LP loaded yet); on
// failure returns nullptr and sets *st and *err
psl_presolver* engine_new(const psl_settings* s, int32_t cap_m, int32_t cap_n, int64_t cap_nnz, int32_t cap_K,
                          psl_status* st, std::string* err);
void engine_free(psl_presolver* p);
// load k LPs (totals within the capacity) and run them
psl_status engine_load(psl_presolver* p, int32_t k, const psl_lp* lps);
psl_status engine_run(psl_presolver* p, psl_stats* out);
// the same run one unit at a time: start, then launch / complete until
// *done (the statistics then as engine_run gives them)
psl_status engine_start(psl_presolver* p);
psl_status engine_launch(psl_presolver* p);
psl_status engine_complete(psl_presolver* p, bool* done);
psl_result engine_result(const psl_presolver* p, int k);
bool engine_has_reduced(const psl_presolver* p, int k);
psl_reduced_view engine_view(const psl_presolver* p, int k);
// LP k's records of the last run: count, and their device address
int64_t engine_records(const psl_presolver* p, int k, const void** dev);
const std::string& engine_error(const psl_presolver* p);
int32_t engine_error_lp(const psl_presolver* p);
// per-LP statistics of the last run (as psl_batch_stats)
void engine_lp_stats(const psl_presolver* p, int k, psl_stats* out);
// the original LP by rows, on the host: row i's columns in ci[rp[i]..rp[i+1])
// with values va (free-singleton records take x_j from their row)
struct HostRows {
  std::vector<int32_t> rp, ci;
  std::vector<double> va;
};
// true when a record needs the original rows in primal postsolve
bool records_need_rows(const psl_record* rec, int64_t count);
// primal postsolve on the host from records and the reduced column map; rows
// may be null when records_need_rows is false (else PSL_ERR_UNSUPPORTED)
psl_status postsolve_primal(const psl_record* rec, int64_t count, const int32_t* col_map_dev, int32_t n,
                            int32_t n_red, const double* x_red, double* x, const HostRows* rows, double inf_value,
                            std::string* err);
// the original LP by columns, on the host, for dual postsolve: column j's
// rows ascending in ri[cp[j]..cp[j+1]) with values cva, and the costs c
struct HostCols {
  std::vector<int32_t> cp, ri;
  std::vector<double> cva, c;
};
// dual postsolve on the host (row duals y[m], reduced costs z[n] of the
// original LP from the reduced problem's row duals y_red[m_red])
void postsolve_dual(const psl_record* rec, int64_t count, int32_t m, int32_t n, const std::vector<int32_t>& row_map,
                    const double* y_red, const HostCols& A, double* y, double* z);
size_t engine_arena_bytes(const psl_presolver* p);
// the message psl_last_error(NULL) returns on this thread
void set_create_error(const std::string& msg);
// one presolve in static scratch (psl_presolve_noalloc's work): device arrays
// carved from dev_scratch, host staging from host_stage, the 8 events given
psl_status engine_run_static(const psl_lp* lp, const psl_settings* s, unsigned char* dev_scratch, size_t dev_bytes,
                             unsigned char* host_stage, size_t host_bytes, hipEvent_t* ev, psl_noalloc_out* out,
                             psl_result* res, psl_stats* stats, std::string* err);
// LP k's original rows / columns on the host (after a run; for postsolve)
psl_status engine_host_rows(psl_presolver* p, int k, HostRows& A);
psl_status engine_host_cols(psl_presolver* p, int k, HostCols& A);

}  // namespace psl
