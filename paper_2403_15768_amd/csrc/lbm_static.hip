// lbm_static.hip -- the friction quadrature for callers that cannot allocate.
//
// lbm_friction_quadrature_static() runs the same kernels as
// lbm_set_friction_spectral() (k_friction_raw / k_friction_full, then the
// normalisation k_friction_lat) on caller-owned device arrays, with no
// context and no device allocation: the raw quadrature sums, which the
// normalisation needs and the context keeps in its arena, live in a
// file-scope device array of fixed size instead.  Each GPU holds its own
// copy of that array until the process ends.  The host never passes the
// array's name to a kernel (in host code it is a stand-in, not a device
// address): the device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm_internal.h"

// raw sums of at most kStaticMaxNodes wall nodes plus the reference (8 MiB)
constexpr size_t kStaticMaxNodes = LBM_STATIC_MAX_NODES;

static __device__ __align__(256) double scratch[kStaticMaxNodes + 1];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// the current device's copy of `scratch` (looked up on the first call there)
lbm_status scratch_ptr(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LBM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return LBM_EDEVICE;
    }
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_friction_quadrature_static(const lbm_spectral* sp, const double* omega, size_t n,
                                          double* lambda, void* hip_stream) {
  if (!lbm_host::spectral_valid(sp)) return LBM_EINVAL;
  if (n > kStaticMaxNodes) return LBM_EINVAL;
  if (n > 0 && (!omega || !lambda)) return LBM_EINVAL;
  double* raw = nullptr;
  lbm_status s = scratch_ptr(&raw);
  if (s != LBM_OK) return s;
  // every raw sum the normalisation reads (k <= n) is written first by the
  // quadrature kernel on the same stream: nothing needs clearing
  const hipError_t e = lbm::launch_friction(lbm_host::spec_args(sp), omega, (int64_t)n, raw,
                                            lambda, reinterpret_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

}  // extern "C"
