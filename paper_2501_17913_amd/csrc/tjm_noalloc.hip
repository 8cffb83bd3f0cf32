// The truncated SVD building block with no allocation: the same kernel as
// tjm_selftest_svd, on caller-provided device buffers, with its work arrays
// in a fixed device array of this library.  For callers that cannot call
// hipMalloc (graph capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <mutex>

#include "tjm_internal.h"
#include "tjm_selftest.h"

namespace {
// Largest working set: the rotated matrix is p x nc with p <= 256 rows and
// nc <= 128 columns; the three work arrays (Wc and Uc: p x nc, Tg: m x n
// <= 128 x 256) each hold at most this many complex doubles.
constexpr long kWorkComplex = 256L * 128L;
constexpr int kMaxDevices = 64;
}  // namespace

// 3 x 32768 complex doubles = 1.5 MiB per device, held until the process ends
static __device__ __align__(256) double scratch[3 * 2 * kWorkComplex];

namespace {
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};   // device address of scratch, per device ordinal
}  // namespace

// Device address of scratch on the current device, looked up once per device.
static tjm_status scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return tjm_fail_global(TJM_E_DEVICE, "no current HIP device");
  if (dev >= kMaxDevices) return tjm_fail_global(TJM_E_UNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return tjm_fail_global(TJM_E_DEVICE, "hipGetSymbolAddress(scratch) failed");
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return TJM_OK;
}

extern "C" tjm_status tjm_svd_noalloc(int m, int n, const double* G, double discard, int cap, double deg_tol,
                                      int absorb_left, double* left, double* right, double* S, int* k,
                                      void* stream) {
  if (m < 1 || n < 1 || cap < 1) return tjm_fail_global(TJM_E_INVAL, "svd_noalloc: m, n and cap must be >= 1");
  if ((absorb_left ? m : n) > 128 || (m > n ? m : n) > 256)
    return tjm_fail_global(TJM_E_INVAL,
                           "svd_noalloc: needs max(m, n) <= 256 and n <= 128 (m <= 128 with absorb_left), "
                           "the size of its fixed work arrays");
  if (!G || !left || !right || !S || !k) return tjm_fail_global(TJM_E_INVAL, "svd_noalloc: NULL buffer");
  double* ws = nullptr;
  const tjm_status st = scratch_on_current_device(&ws);
  if (st != TJM_OK) return st;
  double* Wc = ws;
  double* Uc = ws + 2 * kWorkComplex;
  double* Tg = ws + 4 * kWorkComplex;
  const hipError_t e = tjm_launch_st_svd(m, n, G, discard, cap, deg_tol, absorb_left, left, right, S, k, Wc, Uc,
                                         Tg, (hipStream_t)stream);
  if (e != hipSuccess) return tjm_fail_global(TJM_E_DEVICE, hipGetErrorString(e));
  return TJM_OK;
}
