// gather_probe.hip -- libpsl_probe.so: the rate at which this GPU serves
// random 16-byte gathers from a table too large for its caches, beside a
// streamed 12-byte index + coefficient per gather. This is the access
// pattern of the row sweep (the bounds of each entry's column, gathered in
// the order the rows store their columns), so it is the practical ceiling of
// the sweep's gathers, well below the HBM peak: every gather moves a whole
// line for 16 useful bytes. A measurement helper, not part of libpsl.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_probe_init(uint32_t* idx, double* va, int64_t n, uint64_t entries, double2* tab) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    idx[i] = (uint32_t)(mix64((uint64_t)i) % entries);
    va[i] = 1.0;
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)entries; t += stride)
    tab[t] = make_double2((double)t, 1.0);
}

// four gathers in flight per lane, as the sweep issues a row block's loads
__global__ void __launch_bounds__(256) k_probe_gather(const uint32_t* idx, const double* va, const double2* tab,
                                                       int64_t n, double* out) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double s = 0.0;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += 4 * stride) {
    uint32_t j[4];
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int64_t i = i0 + u * stride;
      j[u] = i < n ? idx[i] : 0u;
      a[u] = i < n ? va[i] : 0.0;
    }
    double2 b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) b[u] = tab[j[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) s = s + a[u] * (b[u].x + b[u].y);
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// Random 16-byte gathers per second (best of reps launches of n gathers
// from a table of `entries` 16-byte elements, uniformly random indices).
// Allocates and frees its own device memory. Returns 0, or -1 on a HIP error
// or invalid sizes (entries must be in [1, 2^32), n >= 1, reps >= 1).
extern "C" int psl_probe_gather(int64_t entries, int64_t n, int32_t reps, double* gathers_per_s) {
  if (entries < 1 || entries >= (1ll << 32) || n < 1 || reps < 1 || !gathers_per_s) return -1;
  const int grid = 8192;
  uint32_t* idx = nullptr;
  double* va = nullptr;
  double2* tab = nullptr;
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -1;
  float best = 0.0f;
  if (hipMalloc(&idx, (size_t)n * 4) != hipSuccess) goto done;
  if (hipMalloc(&va, (size_t)n * 8) != hipSuccess) goto done;
  if (hipMalloc(&tab, (size_t)entries * 16) != hipSuccess) goto done;
  if (hipMalloc(&out, (size_t)grid * 256 * 8) != hipSuccess) goto done;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  hipLaunchKernelGGL(k_probe_init, dim3(grid), dim3(256), 0, 0, idx, va, n, (uint64_t)entries, tab);
  for (int r = 0; r <= reps; ++r) {
    if (hipEventRecord(e0, 0) != hipSuccess) goto done;
    hipLaunchKernelGGL(k_probe_gather, dim3(grid), dim3(256), 0, 0, idx, va, tab, n, out);
    if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) goto done;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) goto done;
    if (r > 0 && (best == 0.0f || ms < best)) best = ms;  // the first launch warms up
  }
  if (hipGetLastError() != hipSuccess || best <= 0.0f) goto done;
  *gathers_per_s = (double)n / (best * 1e-3);
  rc = 0;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (idx) (void)hipFree(idx);
  if (va) (void)hipFree(va);
  if (tab) (void)hipFree(tab);
  if (out) (void)hipFree(out);
  return rc;
}
