// server.hip -- serving: continuous batching of a stream of LPs.
//
// Requests wait in a FIFO queue. A slot (a batch engine with its own arena,
// stream and, in threaded mode, worker thread) takes every waiting LP from
// the head of the queue that fits its capacity and whose reduced problem can
// be reserved in the result heap, presolves them as one batch (every LP gets
// its alone result), then copies each reduced problem into its reserved block
// with one scatter-copy launch and the records to the host. Slots run
// concurrently, so requests that arrive while a batch is on the device start
// on another slot as soon as it is free. The result heap is the device-memory
// budget left after the arenas; a block stays allocated until its ticket is
// released, and the head of the queue waits while its reservation does not
// fit (admission by HBM footprint, no overtaking).
//
// Without worker threads the server is stepped: each psl_server_step admits
// waiting LPs into the free slots, advances every resident batch by one unit
// of its run (a propagation round, a cycle's reduction pass, or the
// compaction; all slots' launches before any wait, so their streams overlap)
// and retires the batches whose run ended.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

using namespace psl;

namespace {

using Clock = std::chrono::steady_clock;

thread_local std::string g_server_error = "no error";

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// first-fit allocator over one device allocation (offsets only)
// ---------------------------------------------------------------------------
class Heap {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(std::max<size_t>(bytes, 256));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      size_t rest = it->second - bytes;
      size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(std::max<size_t>(bytes, 256));
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  // keep the first new_bytes of a block of old_bytes
  void shrink(size_t off, size_t old_bytes, size_t new_bytes) {
    old_bytes = align256(std::max<size_t>(old_bytes, 256));
    new_bytes = align256(std::max<size_t>(new_bytes, 256));
    if (new_bytes < old_bytes) release(off + new_bytes, old_bytes - new_bytes);
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0, peak_ = 0;
};

// the arrays of a reduced problem, laid out in one heap block
struct Layout {
  size_t off[15];
  size_t total;
};

Layout layout_of(int64_t m, int64_t n, int64_t nnz) {
  const size_t sz[15] = {(size_t)(m + 1) * 4, (size_t)nnz * 4, (size_t)nnz * 8, (size_t)(n + 1) * 4,
                         (size_t)nnz * 4,     (size_t)nnz * 8, (size_t)m * 8,   (size_t)m * 8,
                         (size_t)n * 8,       (size_t)n * 8,   (size_t)n * 8,   (size_t)m * 4,
                         (size_t)n * 4,       (size_t)m,       (size_t)n};
  Layout L;
  size_t at = 0;
  for (int a = 0; a < 15; ++a) {
    L.off[a] = at;
    at += align256(sz[a]);
  }
  L.total = at;
  return L;
}

// ---------------------------------------------------------------------------
// scatter copy: many (src, dst, bytes) segments in one launch
// ---------------------------------------------------------------------------
struct CopySeg {
  const char* src;
  char* dst;
  int64_t bytes;
  int64_t chunk0;  // first chunk of this segment
};

#define COPY_CHUNK 16384

__global__ void __launch_bounds__(256) k_copy_segs(const CopySeg* segs, int nseg) {
  int64_t c = blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[mid].chunk0 <= c) lo = mid;
    else hi = mid - 1;
  }
  CopySeg sg = segs[lo];
  int64_t o0 = (c - sg.chunk0) * COPY_CHUNK;
  int64_t o1 = o0 + COPY_CHUNK < sg.bytes ? o0 + COPY_CHUNK : sg.bytes;
  bool words = ((uintptr_t)sg.src % 4 == 0) && ((uintptr_t)sg.dst % 4 == 0) && (sg.bytes % 4 == 0);
  if (words) {
    const uint32_t* s = (const uint32_t*)(sg.src + o0);
    uint32_t* d = (uint32_t*)(sg.dst + o0);
    int64_t nw = (o1 - o0) / 4;
    for (int64_t w = threadIdx.x; w < nw; w += blockDim.x) d[w] = s[w];
  } else {
    for (int64_t b = o0 + threadIdx.x; b < o1; b += blockDim.x) sg.dst[b] = sg.src[b];
  }
}

enum : int { T_QUEUED = 0, T_RUNNING = 1, T_DONE = 2 };

struct Ticket {
  uint64_t id = 0;
  psl_lp lp{};
  int state = T_QUEUED;
  Clock::time_point arrival, start, done;
  size_t heap_off = 0, heap_bytes = 0;
  bool has_block = false;
  psl_ticket_info info{};
  psl_reduced_view view{};
  std::vector<psl_record> records;
  std::string err;
  bool kept = false;     // keep_original: the LP's rows and columns on the host
  HostRows rows;
  HostCols cols;
};

struct Slot {
  int index = 0;
  psl_presolver* eng = nullptr;
  hipStream_t stream = nullptr;
  CopySeg* segs_dev = nullptr;
  CopySeg* segs_host = nullptr;  // pinned
  int64_t seg_cap = 0;
  std::vector<psl_record> rec_host;
  std::thread th;
  // stepped server: the batch resident on the slot (its tickets, and those
  // loaded) while its run goes unit by unit
  bool busy = false;
  std::vector<Ticket*> batch, live;
};

}  // namespace

struct psl_server {
  psl_server_config cfg{};
  psl_settings s{};
  std::mutex mu;
  std::mutex step_mu;  // stepped server: one step at a time (the slots' state)
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
  std::deque<uint64_t> unpolled;
  uint64_t next_id = 1;
  Heap heap;
  char* heap_mem = nullptr;
  std::vector<std::unique_ptr<Slot>> slots;
  bool stop = false;
  int running = 0;
  size_t arena_bytes = 0;
  std::string err = "no error";
};

extern "C" void psl_server_config_default(psl_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->hbm_budget_bytes = (size_t)64 << 30;
  c->slots = 4;
  c->threaded = 1;
  c->max_batch_lps = 1024;
  c->max_batch_rows = 2600000;
  c->max_batch_cols = 3900000;
  c->max_batch_nnz = 30000000;
  c->keep_original = 0;
}

static size_t footprint(const psl_lp& lp) { return layout_of(lp.m, lp.n, lp.nnz).total; }

// LPs from the head of the queue for one batch (lock held): capacity of the
// slot, same memory kind as the head, and a heap block for each
static std::vector<Ticket*> take_batch(psl_server* sv) {
  std::vector<Ticket*> b;
  int64_t M = 0, Nc = 0, Z = 0;
  const psl_server_config& c = sv->cfg;
  while (!sv->queue.empty() && (int32_t)b.size() < c.max_batch_lps) {
    Ticket* t = sv->tickets[sv->queue.front()].get();
    const psl_lp& lp = t->lp;
    if (!b.empty() && lp.mem != b[0]->lp.mem) break;
    if (M + lp.m > c.max_batch_rows || Nc + lp.n > c.max_batch_cols || Z + lp.nnz > c.max_batch_nnz) break;
    size_t off = 0, need = footprint(lp);
    if (!sv->heap.alloc(need, &off)) break;
    t->heap_off = off;
    t->heap_bytes = need;
    t->has_block = true;
    t->state = T_RUNNING;
    t->start = Clock::now();
    sv->queue.pop_front();
    b.push_back(t);
    M += lp.m;
    Nc += lp.n;
    Z += lp.nnz;
  }
  return b;
}

// results of a batch become visible (lock held)
static void publish(psl_server* sv, Slot& sl, std::vector<Ticket*>& b) {
  Clock::time_point now = Clock::now();
  for (Ticket* t : b) {
    t->done = now;
    t->state = T_DONE;
    t->info.queue_ms = ms_between(t->arrival, t->start);
    t->info.latency_ms = ms_between(t->arrival, t->done);
    t->info.batch_lps = (int32_t)b.size();
    t->info.slot = sl.index;
    if (t->has_block && t->view.row_ptr == nullptr) {  // no reduced problem to keep
      sv->heap.release(t->heap_off, t->heap_bytes);
      t->has_block = false;
    }
    sv->unpolled.push_back(t->id);
  }
  sv->cv_done.notify_all();
  sv->cv_work.notify_all();
}

static void fail_ticket(Ticket* t, psl_status st, const std::string& msg) {
  t->info.status = st;
  t->err = msg;
  t->view = psl_reduced_view{};
}

// load a batch's LPs on a slot's engine (lock not held): an invalid LP fails
// its ticket and the others are loaded again; live = the loaded tickets
// (empty when none is left)
static psl_status load_batch(Slot& sl, const std::vector<Ticket*>& b, std::vector<Ticket*>& live) {
  live = b;
  std::vector<psl_lp> lps;
  psl_status st = PSL_OK;
  for (;;) {
    lps.clear();
    for (Ticket* t : live) lps.push_back(t->lp);
    if (lps.empty()) return PSL_OK;
    st = engine_load(sl.eng, (int32_t)lps.size(), lps.data());
    if (st == PSL_ERR_INVALID && engine_error_lp(sl.eng) >= 0 && engine_error_lp(sl.eng) < (int)live.size()) {
      // drop the invalid LP and load the others again
      int bad = engine_error_lp(sl.eng);
      fail_ticket(live[bad], st, engine_error(sl.eng));
      live.erase(live.begin() + bad);
      continue;
    }
    break;
  }
  if (st != PSL_OK) {
    for (Ticket* t : live) fail_ticket(t, st, engine_error(sl.eng));
    live.clear();
  }
  return st;
}

static void finish_batch(psl_server* sv, Slot& sl, std::vector<Ticket*>& live);

// presolve one batch on a slot and copy its results out (lock not held)
static void run_batch(psl_server* sv, Slot& sl, std::vector<Ticket*>& b) {
  std::vector<Ticket*> live;
  if (load_batch(sl, b, live) != PSL_OK || live.empty()) return;
  psl_stats S{};
  psl_status st = engine_run(sl.eng, &S);
  if (st != PSL_OK) {
    for (Ticket* t : live) fail_ticket(t, st, engine_error(sl.eng));
    return;
  }
  finish_batch(sv, sl, live);
}

// after a batch's run: its reduced problems into their heap blocks, its
// records to the host (lock not held)
static void finish_batch(psl_server* sv, Slot& sl, std::vector<Ticket*>& live) {
  // reduced problems into their blocks, records to the host
  int64_t nseg = 0, chunks = 0, total_rec = 0;
  const void* rec0 = nullptr;
  std::vector<int64_t> rec_at(live.size());
  for (size_t k = 0; k < live.size(); ++k) {
    Ticket* t = live[k];
    t->info.status = PSL_OK;
    t->info.result = engine_result(sl.eng, (int)k);
    engine_lp_stats(sl.eng, (int)k, &t->info.stats);
    const void* dev = nullptr;
    int64_t cnt = engine_records(sl.eng, (int)k, &dev);
    if (k == 0) rec0 = dev;
    rec_at[k] = total_rec;
    t->records.resize((size_t)cnt);
    total_rec += cnt;
    t->view = psl_reduced_view{};
    if (!engine_has_reduced(sl.eng, (int)k)) continue;
    psl_reduced_view v = engine_view(sl.eng, (int)k);
    Layout L = layout_of(v.m, v.n, v.nnz);
    char* base = sv->heap_mem + t->heap_off;
    const void* srcs[15] = {v.row_ptr, v.col_idx, v.val, v.col_ptr, v.row_idx, v.cval, v.lhs, v.rhs,
                            v.lb,      v.ub,      v.c,   v.row_map, v.col_map, v.row_class, v.col_class};
    const size_t sz[15] = {(size_t)(v.m + 1) * 4, (size_t)v.nnz * 4, (size_t)v.nnz * 8, (size_t)(v.n + 1) * 4,
                           (size_t)v.nnz * 4,     (size_t)v.nnz * 8, (size_t)v.m * 8,   (size_t)v.m * 8,
                           (size_t)v.n * 8,       (size_t)v.n * 8,   (size_t)v.n * 8,   (size_t)v.m * 4,
                           (size_t)v.n * 4,       (size_t)v.m,       (size_t)v.n};
    for (int a = 0; a < 15; ++a) {
      if (sz[a] == 0) continue;
      if (nseg >= sl.seg_cap) break;  // never: 15 per LP are reserved
      CopySeg& g = sl.segs_host[nseg++];
      g.src = (const char*)srcs[a];
      g.dst = base + L.off[a];
      g.bytes = (int64_t)sz[a];
      g.chunk0 = chunks;
      chunks += (g.bytes + COPY_CHUNK - 1) / COPY_CHUNK;
    }
    psl_reduced_view& o = t->view;
    o = v;
    o.row_ptr = (const int32_t*)(base + L.off[0]);
    o.col_idx = (const int32_t*)(base + L.off[1]);
    o.val = (const double*)(base + L.off[2]);
    o.col_ptr = (const int32_t*)(base + L.off[3]);
    o.row_idx = (const int32_t*)(base + L.off[4]);
    o.cval = (const double*)(base + L.off[5]);
    o.lhs = (const double*)(base + L.off[6]);
    o.rhs = (const double*)(base + L.off[7]);
    o.lb = (const double*)(base + L.off[8]);
    o.ub = (const double*)(base + L.off[9]);
    o.c = (const double*)(base + L.off[10]);
    o.row_map = (const int32_t*)(base + L.off[11]);
    o.col_map = (const int32_t*)(base + L.off[12]);
    o.row_class = (const uint8_t*)(base + L.off[13]);
    o.col_class = (const uint8_t*)(base + L.off[14]);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->heap.shrink(t->heap_off, t->heap_bytes, L.total);
      t->heap_bytes = align256(std::max<size_t>(L.total, 256));
    }
  }
  hipError_t e = hipSuccess;
  if (nseg > 0) {
    e = hipMemcpyAsync(sl.segs_dev, sl.segs_host, nseg * sizeof(CopySeg), hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_copy_segs, dim3((unsigned)chunks), dim3(256), 0, sl.stream, (const CopySeg*)sl.segs_dev,
                         (int)nseg);
      e = hipGetLastError();
    }
  }
  // the records of all LPs of the batch are contiguous (split by LP)
  if (e == hipSuccess && total_rec > 0) {
    sl.rec_host.resize((size_t)total_rec);
    e = hipMemcpyAsync(sl.rec_host.data(), rec0, total_rec * sizeof(psl_record), hipMemcpyDeviceToHost, sl.stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
  if (e != hipSuccess) {
    for (Ticket* t : live) fail_ticket(t, PSL_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
    return;
  }
  for (size_t k = 0; k < live.size(); ++k)
    if (!live[k]->records.empty())
      std::memcpy(live[k]->records.data(), sl.rec_host.data() + rec_at[k],
                  live[k]->records.size() * sizeof(psl_record));
  // keep_original: the LPs' rows and columns, for postsolves that need them
  if (sv->cfg.keep_original) {
    for (size_t k = 0; k < live.size(); ++k) {
      Ticket* t = live[k];
      if (!t->has_block) continue;
      psl_status s1 = engine_host_rows(sl.eng, (int)k, t->rows);
      if (s1 == PSL_OK) s1 = engine_host_cols(sl.eng, (int)k, t->cols);
      if (s1 != PSL_OK) {
        fail_ticket(t, s1, engine_error(sl.eng));
        continue;
      }
      t->kept = true;
    }
  }
}

static void worker(psl_server* sv, Slot* sl) {
  (void)hipSetDevice(sv->s.device);
  for (;;) {
    std::vector<Ticket*> b;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      for (;;) {
        if (sv->stop) return;
        b = take_batch(sv);
        if (!b.empty()) break;
        sv->cv_work.wait(lk);
      }
      ++sv->running;
    }
    run_batch(sv, *sl, b);
    std::lock_guard<std::mutex> lk(sv->mu);
    --sv->running;
    publish(sv, *sl, b);
  }
}

static void destroy(psl_server* sv) {
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto& sl : sv->slots)
    if (sl->th.joinable()) sl->th.join();
  (void)hipSetDevice(sv->s.device);
  for (auto& sl : sv->slots) {
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    if (sl->eng) engine_free(sl->eng);
    if (sl->segs_dev) (void)hipFree(sl->segs_dev);
    if (sl->segs_host) (void)hipHostFree(sl->segs_host);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
  }
  if (sv->heap_mem) (void)hipFree(sv->heap_mem);
  delete sv;
}

extern "C" psl_status psl_server_create(const psl_server_config* c, const psl_settings* s, psl_server** out) {
  if (!c || !out) {
    g_server_error = "null argument";
    return PSL_ERR_INVALID;
  }
  psl_settings def;
  psl_settings_default(&def);
  if (!s) s = &def;
  std::string e = check_settings(s);
  if (e.empty() && (c->slots < 1 || c->slots > 16)) e = "slots must be in [1, 16]";
  if (e.empty() && (c->max_batch_lps < 1 || c->max_batch_rows < 1 || c->max_batch_cols < 1 ||
                    c->max_batch_nnz < 1 || c->max_batch_nnz >= ((int64_t)1 << 30)))
    e = "batch limits must be positive (nnz below 2^30)";
  if (!e.empty()) {
    g_server_error = e;
    return PSL_ERR_INVALID;
  }
  if (s->device_records > 0) {
    g_server_error = "device_records (a flushed record stack) is for single-LP presolvers";
    return PSL_ERR_UNSUPPORTED;
  }
  if (hipSetDevice(s->device) != hipSuccess) {
    g_server_error = "cannot select the device";
    return PSL_ERR_DEVICE;
  }
  psl_server* sv = new psl_server();
  sv->cfg = *c;
  sv->s = *s;
  sv->s.bin_thresholds = nullptr;  // the engines copy the thresholds at creation
  size_t arenas = 0;
  for (int k = 0; k < c->slots; ++k) {
    auto sl = std::make_unique<Slot>();
    sl->index = k;
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      g_server_error = "cannot create a stream";
      sv->slots.push_back(std::move(sl));
      destroy(sv);
      return PSL_ERR_DEVICE;
    }
    psl_settings es = *s;
    es.stream = sl->stream;
    psl_status st = PSL_OK;
    std::string err;
    sl->eng = engine_new(&es, c->max_batch_rows, c->max_batch_cols, c->max_batch_nnz, c->max_batch_lps, &st, &err);
    sl->seg_cap = 15 * (int64_t)c->max_batch_lps;
    bool ok = sl->eng != nullptr;
    if (ok) ok = hipMalloc((void**)&sl->segs_dev, sl->seg_cap * sizeof(CopySeg)) == hipSuccess;
    if (ok) ok = hipHostMalloc((void**)&sl->segs_host, sl->seg_cap * sizeof(CopySeg), hipHostMallocDefault) == hipSuccess;
    if (sl->eng) arenas += engine_arena_bytes(sl->eng) + sl->seg_cap * sizeof(CopySeg);
    sv->slots.push_back(std::move(sl));
    if (!ok) {
      g_server_error = sv->slots.back()->eng ? "cannot allocate the copy descriptors" : err;
      destroy(sv);
      return st != PSL_OK ? st : PSL_ERR_OOM;
    }
  }
  if (arenas >= c->hbm_budget_bytes) {
    g_server_error = "the budget does not cover the slot arenas (" + std::to_string(arenas) + " bytes)";
    destroy(sv);
    return PSL_ERR_CAPACITY;
  }
  sv->arena_bytes = arenas;
  size_t heap = (c->hbm_budget_bytes - arenas) & ~(size_t)255;
  if (hipMalloc((void**)&sv->heap_mem, heap) != hipSuccess) {
    (void)hipGetLastError();
    g_server_error = "cannot allocate the result heap of " + std::to_string(heap) + " bytes";
    destroy(sv);
    return PSL_ERR_OOM;
  }
  sv->heap.init(heap);
  if (c->threaded)
    for (auto& sl : sv->slots) sl->th = std::thread(worker, sv, sl.get());
  *out = sv;
  return PSL_OK;
}

static psl_status sfail(psl_server* sv, psl_status st, const std::string& msg) {
  sv->err = msg;
  return st;
}

extern "C" psl_status psl_server_submit(psl_server* sv, const psl_lp* lp, uint64_t* ticket) {
  if (!sv || !lp || !ticket) return PSL_ERR_INVALID;
  std::string e = check_lp_shape(lp);
  if (!e.empty()) return sfail(sv, PSL_ERR_INVALID, e);
  const psl_server_config& c = sv->cfg;
  if (lp->m > c.max_batch_rows || lp->n > c.max_batch_cols || lp->nnz > c.max_batch_nnz)
    return sfail(sv, PSL_ERR_CAPACITY, "the LP exceeds the batch capacity");
  if (align256(footprint(*lp)) > sv->heap.size())
    return sfail(sv, PSL_ERR_CAPACITY, "the LP's reduced problem cannot fit the result heap");
  auto t = std::make_unique<Ticket>();
  t->lp = *lp;
  t->arrival = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  t->id = sv->next_id++;
  *ticket = t->id;
  sv->queue.push_back(t->id);
  sv->tickets.emplace(t->id, std::move(t));
  sv->cv_work.notify_one();
  return PSL_OK;
}

// the batch on a stepped slot ended, or failed with st (lock not held)
static void retire(psl_server* sv, Slot& sl, psl_status st) {
  if (st != PSL_OK) {
    for (Ticket* t : sl.live) fail_ticket(t, st, engine_error(sl.eng));
  } else if (!sl.live.empty()) {
    finish_batch(sv, sl, sl.live);
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  --sv->running;
  publish(sv, sl, sl.batch);
  sl.busy = false;
  sl.batch.clear();
  sl.live.clear();
}

extern "C" psl_status psl_server_step(psl_server* sv, int32_t* n_run) {
  if (!sv || !n_run) return PSL_ERR_INVALID;
  if (sv->cfg.threaded) return sfail(sv, PSL_ERR_STATE, "the server runs its own worker threads");
  std::lock_guard<std::mutex> step_lock(sv->step_mu);
  (void)hipSetDevice(sv->s.device);
  // admit: every free slot takes the next batch from the queue head
  for (auto& slp : sv->slots) {
    Slot& sl = *slp;
    if (sl.busy) continue;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sl.batch = take_batch(sv);
      if (sl.batch.empty()) break;  // nothing waiting, or the head does not fit yet
      ++sv->running;
    }
    sl.busy = true;
    psl_status st = load_batch(sl, sl.batch, sl.live);
    if (st == PSL_OK && !sl.live.empty()) st = engine_start(sl.eng);
    if (st != PSL_OK || sl.live.empty()) retire(sv, sl, st);
  }
  // one unit (a round, a cycle's reduction pass or the compaction) of every
  // resident batch: all launches first, so the slots' streams overlap
  int32_t advanced = 0;
  for (auto& slp : sv->slots) {
    Slot& sl = *slp;
    if (!sl.busy) continue;
    advanced += (int32_t)sl.live.size();
    psl_status st = engine_launch(sl.eng);
    if (st != PSL_OK) retire(sv, sl, st);
  }
  // then the completions; a batch whose run ended is retired
  for (auto& slp : sv->slots) {
    Slot& sl = *slp;
    if (!sl.busy) continue;
    bool done = false;
    psl_status st = engine_complete(sl.eng, &done);
    if (st != PSL_OK || done) retire(sv, sl, st);
  }
  *n_run = advanced;
  return PSL_OK;
}

extern "C" psl_status psl_server_poll(psl_server* sv, uint64_t* tickets, int32_t cap, int32_t* n_done) {
  if (!sv || !n_done || (cap > 0 && !tickets)) return PSL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  int32_t k = 0;
  while (k < cap && !sv->unpolled.empty()) {
    tickets[k++] = sv->unpolled.front();
    sv->unpolled.pop_front();
  }
  *n_done = k;
  return PSL_OK;
}

static Ticket* find_ticket(psl_server* sv, uint64_t id) {
  auto it = sv->tickets.find(id);
  return it == sv->tickets.end() ? nullptr : it->second.get();
}

extern "C" psl_status psl_server_wait(psl_server* sv, uint64_t ticket, double timeout_ms) {
  if (!sv) return PSL_ERR_INVALID;
  std::unique_lock<std::mutex> lk(sv->mu);
  Ticket* t = find_ticket(sv, ticket);
  if (!t) return sfail(sv, PSL_ERR_INVALID, "unknown ticket");
  auto pred = [&] { return t->state == T_DONE; };
  if (timeout_ms < 0) {
    sv->cv_done.wait(lk, pred);
  } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred)) {
    sv->err = "timed out waiting for the ticket";
    return PSL_ERR_STATE;
  }
  return PSL_OK;
}

// a done ticket (lock held)
static psl_status done_ticket(psl_server* sv, uint64_t id, Ticket** out) {
  Ticket* t = find_ticket(sv, id);
  if (!t) return sfail(sv, PSL_ERR_INVALID, "unknown ticket");
  if (t->state != T_DONE) return sfail(sv, PSL_ERR_STATE, "the ticket is not done");
  *out = t;
  return PSL_OK;
}

extern "C" psl_status psl_server_info(psl_server* sv, uint64_t ticket, psl_ticket_info* out) {
  if (!sv || !out) return PSL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  Ticket* t = nullptr;
  psl_status st = done_ticket(sv, ticket, &t);
  if (st != PSL_OK) return st;
  *out = t->info;
  return PSL_OK;
}

extern "C" psl_status psl_server_reduced_problem(psl_server* sv, uint64_t ticket, psl_reduced_view* out) {
  if (!sv || !out) return PSL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  Ticket* t = nullptr;
  psl_status st = done_ticket(sv, ticket, &t);
  if (st != PSL_OK) return st;
  if (t->info.status != PSL_OK) return sfail(sv, t->info.status, t->err);
  if (!t->has_block) return sfail(sv, PSL_ERR_STATE, "no reduced problem (infeasible or unbounded LP)");
  *out = t->view;
  return PSL_OK;
}

extern "C" psl_status psl_server_records(psl_server* sv, uint64_t ticket, int64_t* count, psl_record* out,
                                         int64_t cap) {
  if (!sv || !count) return PSL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  Ticket* t = nullptr;
  psl_status st = done_ticket(sv, ticket, &t);
  if (st != PSL_OK) return st;
  if (t->info.status != PSL_OK) return sfail(sv, t->info.status, t->err);
  int64_t c = (int64_t)t->records.size();
  if (out) {
    if (cap < c) return sfail(sv, PSL_ERR_CAPACITY, "record buffer too small");
    if (c) std::memcpy(out, t->records.data(), c * sizeof(psl_record));
  }
  *count = c;
  return PSL_OK;
}

extern "C" psl_status psl_server_postsolve(psl_server* sv, uint64_t ticket, const double* x_red, const double* y_red,
                                           const double* z_red, double* x, double* y, double* z) {
  (void)z_red;  // reduced costs follow from the row duals
  if (!sv) return PSL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  Ticket* t = nullptr;
  psl_status st = done_ticket(sv, ticket, &t);
  if (st != PSL_OK) return st;
  if (t->info.status != PSL_OK) return sfail(sv, t->info.status, t->err);
  if (!t->has_block) return sfail(sv, PSL_ERR_STATE, "no reduced problem to postsolve");
  if ((t->lp.n > 0 && !x) || (t->view.n > 0 && !x_red)) return sfail(sv, PSL_ERR_INVALID, "null solution array");
  if (y_red && !t->kept)
    return sfail(sv, PSL_ERR_UNSUPPORTED, "dual postsolve needs the original LP: create the server with keep_original");
  if (y_red && ((t->lp.m > 0 && !y) || (t->lp.n > 0 && !z))) return sfail(sv, PSL_ERR_INVALID, "null dual array");
  std::string err;
  // without keep_original a done ticket has no original rows (free-singleton
  // records need them: PSL_ERR_UNSUPPORTED then)
  st = postsolve_primal(t->records.data(), (int64_t)t->records.size(), t->view.col_map, t->lp.n, t->view.n, x_red,
                        x, t->kept ? &t->rows : nullptr, sv->s.inf_value, &err);
  if (st != PSL_OK) {
    sv->err = err;
    return st;
  }
  if (!y_red) return PSL_OK;
  std::vector<int32_t> rmap(t->view.m);
  if (t->view.m && hipMemcpy(rmap.data(), t->view.row_map, t->view.m * sizeof(int32_t), hipMemcpyDeviceToHost) !=
                       hipSuccess)
    return sfail(sv, PSL_ERR_DEVICE, "HIP error copying the row map");
  postsolve_dual(t->records.data(), (int64_t)t->records.size(), t->lp.m, t->lp.n, rmap, y_red, t->cols, y, z);
  return PSL_OK;
}

extern "C" psl_status psl_server_release(psl_server* sv, uint64_t ticket) {
  if (!sv) return PSL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  Ticket* t = nullptr;
  psl_status st = done_ticket(sv, ticket, &t);
  if (st != PSL_OK) return st;
  if (t->has_block) sv->heap.release(t->heap_off, t->heap_bytes);
  sv->tickets.erase(ticket);
  sv->cv_work.notify_all();
  return PSL_OK;
}

extern "C" psl_status psl_server_drain(psl_server* sv) {
  if (!sv) return PSL_ERR_INVALID;
  if (!sv->cfg.threaded) {
    for (;;) {
      int32_t n = 0;
      psl_status st = psl_server_step(sv, &n);
      if (st != PSL_OK) return st;
      if (n > 0) continue;
      std::lock_guard<std::mutex> lk(sv->mu);
      if (sv->queue.empty()) return PSL_OK;
      return sfail(sv, PSL_ERR_CAPACITY, "the queue head does not fit the result heap");
    }
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_done.wait(lk, [&] { return sv->queue.empty() && sv->running == 0; });
  return PSL_OK;
}

extern "C" psl_status psl_server_memory(psl_server* sv, size_t* arena_bytes, size_t* heap_bytes, size_t* heap_used,
                                        size_t* heap_peak) {
  if (!sv || !arena_bytes || !heap_bytes || !heap_used || !heap_peak) return PSL_ERR_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  *arena_bytes = sv->arena_bytes;
  *heap_bytes = sv->heap.size();
  *heap_used = sv->heap.used();
  *heap_peak = sv->heap.peak();
  return PSL_OK;
}

extern "C" void psl_server_free(psl_server* sv) {
  if (sv) destroy(sv);
}

extern "C" const char* psl_server_last_error(const psl_server* sv) {
  if (!sv) return g_server_error.c_str();
  return sv->err.c_str();
}
