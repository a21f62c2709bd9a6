// slm_split_scan_noalloc: the histogram scan of slm_split_scan for callers
// that cannot allocate device memory.  Its accumulator lives in a file-scope
// device array of the library (one copy per GPU, held until the process
// ends) instead of a caller workspace.
#include "slm_internal.hpp"

#include <mutex>

namespace slm {
namespace {

constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;   // 128 MiB per GPU
constexpr int MAX_DEVICES = 64;

// In host code `scratch` names a host-side stand-in, not device memory: only
// the address hipGetSymbolAddress returns for the current device is used.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES];      // device address of each GPU's array
bool g_dirty[MAX_DEVICES];         // a call failed: the array may not be zero

// Device address of this GPU's scratch array, looked up once per device with
// that device current.  The array is cleared with a fill kernel on the
// call's stream at the first call on a device and after a failed call (the
// scan needs a zero accumulator on entry; every completed scan leaves it
// zero again).
slm_status scratch_of_device(int *dev_out, void **out, hipStream_t s) {
  int dev = -1;
  SLM_HIP(hipGetDevice(&dev));
  SLM_CHECK(dev >= 0 && dev < MAX_DEVICES, SLM_E_UNSUPPORTED,
            "slm_split_scan_noalloc: device %d beyond the %d the library tracks", dev,
            MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    SLM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SLM_CHECK(p != nullptr, SLM_E_HIP, "slm_split_scan_noalloc: no device address for scratch");
    g_scratch[dev] = p;
    g_dirty[dev] = true;
  }
  if (g_dirty[dev]) {
    slm_status st = launch_zero_words(static_cast<uint32_t *>(g_scratch[dev]),
                                      (int64_t)(SCRATCH_BYTES / 4), s);
    if (st) return st;
    g_dirty[dev] = false;
  }
  *dev_out = dev;
  *out = g_scratch[dev];
  return SLM_OK;
}

void mark_dirty(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  g_dirty[dev] = true;
}

}  // namespace
}  // namespace slm

using namespace slm;

extern "C" {

size_t slm_split_scan_noalloc_max_bytes(void) { return SCRATCH_BYTES; }

slm_status slm_split_scan_noalloc(const float *Z, int32_t z_layout, const float *zmin,
                                  const float *zmax, const void *target, int32_t t_dtype,
                                  int32_t K, int64_t N, const int64_t *row_off, int32_t n_nodes,
                                  int32_t P, int32_t bins, int32_t crit, int32_t *best_split,
                                  double *best_loss, float *threshold, uint32_t *hist_out,
                                  double *sums_out, void *stream) {
  clear_error();
  SLM_CHECK(bins >= 2 && bins <= 256, SLM_E_UNSUPPORTED,
            "slm_split_scan_noalloc: histogram scans only (bins in 2..256; the exact scan "
            "needs no scratch: use slm_split_scan)");
  SLM_CHECK(N >= 0 && N < (1ll << 31) && P >= 1 && n_nodes >= 0, SLM_E_SHAPE,
            "slm_split_scan_noalloc: bad sizes");
  const size_t need = slm_split_scan_workspace(N, n_nodes, P, bins, K, crit);
  SLM_CHECK(need <= SCRATCH_BYTES, SLM_E_NOMEM,
            "slm_split_scan_noalloc: this scan needs %zu bytes of scratch; the library holds "
            "%zu per GPU",
            need, SCRATCH_BYTES);
  void *ws = nullptr;
  int dev = -1;
  slm_status st = scratch_of_device(&dev, &ws, static_cast<hipStream_t>(stream));
  if (st) return st;
  st = slm_split_scan(Z, z_layout, zmin, zmax, target, t_dtype, K, N, row_off, n_nodes, P, bins,
                      crit, best_split, best_loss, threshold, hist_out, sums_out, ws,
                      SCRATCH_BYTES, stream);
  if (st) mark_dirty(dev);
  return st;
}

}  // extern "C"
