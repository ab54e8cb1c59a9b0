// noalloc.hip -- psl_presolve_noalloc: the presolve of psl_presolve_create +
// psl_presolve_run for callers that cannot allocate device memory. All device
// working memory comes from `scratch`, a static device array of
// PSL_NOALLOC_SCRATCH_BYTES that every device running the library holds
// until the process ends; host staging comes from a static host buffer.
//
// The array's name in host code is a host-side stand-in, not a device
// address: its device address is looked up once per device, with that device
// current, by hipGetSymbolAddress, and only that address is used afterwards
// (kernel arguments, fills, copies).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "engine.h"

namespace {

__device__ __align__(256) unsigned char scratch[PSL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
constexpr size_t kHostStage = 16384;  // the engine's pinned-size host staging for K = 1

struct DeviceScratch {
  std::mutex mu;                 // held for a whole call on the device
  bool ready = false;
  unsigned char* dev = nullptr;  // the device address of `scratch` on this device
  hipEvent_t ev[8] = {nullptr};
  alignas(64) unsigned char host[kHostStage];
};

DeviceScratch g_scratch[kMaxDevices];

// once per device, with the device current: the address of `scratch` there
// and the timing events; returns false with a message on failure
bool set_up(DeviceScratch& ds, std::string* err) {
  if (ds.ready) return true;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    *err = std::string("cannot find the static scratch on the device: ") + hipGetErrorString(e);
    return false;
  }
  for (auto& ev : ds.ev) {
    if (ev) continue;
    e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      *err = std::string("cannot create the scratch's events: ") + hipGetErrorString(e);
      return false;
    }
  }
  ds.dev = (unsigned char*)ptr;
  ds.ready = true;
  return true;
}

psl_status reject(psl_status st, const std::string& msg) {
  psl::set_create_error(msg);
  return st;
}

}  // namespace

extern "C" psl_status psl_presolve_noalloc(const psl_lp* lp, const psl_settings* s, psl_noalloc_out* out,
                                           psl_result* res, psl_stats* stats) {
  if (!lp || !out || !res) return reject(PSL_ERR_INVALID, "null argument");
  psl_settings def;
  psl_settings_default(&def);
  if (!s) s = &def;
  std::string e = psl::check_settings(s);
  if (e.empty()) e = psl::check_lp_shape(lp);
  if (!e.empty()) return reject(PSL_ERR_INVALID, e);
  if (s->device_records > 0)
    return reject(PSL_ERR_UNSUPPORTED, "device_records (a flushed record stack) needs a presolver handle");
  bool rows = lp->m > 0, cols = lp->n > 0, ents = lp->nnz > 0;
  if (!out->row_ptr || !out->col_ptr || (rows && (!out->lhs || !out->rhs || !out->row_map || !out->row_class)) ||
      (cols && (!out->lb || !out->ub || !out->c || !out->col_map || !out->col_class)) ||
      (ents && (!out->col_idx || !out->val || !out->row_idx || !out->cval)) || out->records_cap < 0 ||
      (out->records_cap > 0 && !out->records))
    return reject(PSL_ERR_INVALID, "null output buffer");
  if (s->device < 0 || s->device >= kMaxDevices) return reject(PSL_ERR_INVALID, "device out of range");
  if (hipSetDevice(s->device) != hipSuccess) return reject(PSL_ERR_DEVICE, "cannot select the device");
  DeviceScratch& ds = g_scratch[s->device];
  std::lock_guard<std::mutex> lk(ds.mu);
  if (!set_up(ds, &e)) return reject(PSL_ERR_DEVICE, e);
  psl_status st = psl::engine_run_static(lp, s, ds.dev, PSL_NOALLOC_SCRATCH_BYTES, ds.host, kHostStage, ds.ev, out,
                                         res, stats, &e);
  if (st != PSL_OK) return reject(st, e);
  return PSL_OK;
}
