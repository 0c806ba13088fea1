// Allocation-free variant of the charge-octupole error estimate.
//
// ewald_octupole_error keeps the per-block partial sums of the estimate in a
// plan's workspace.  This variant needs no plan: the partial sums live in a
// fixed array of this library in device memory (`scratch`, one copy per GPU,
// held until the process ends), so the call allocates nothing and suits
// callers that cannot allocate (HIP graph capture, serving loops, harnesses
// that forbid allocation).  The kernels are the plan entry point's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mpewald.h"
#include "ewald_internal.h"

namespace mpe {
ewald_status_t set_error(ewald_status_t st, const char* msg);
void clear_error();
ewald_status_t octupole_args(const double box[3], int n_qm, const double* qm_xyz, const double* omega, int n_mm,
                             const double* mm_xyz, const double* mm_q, int n_r, double r_first, double r_step,
                             double r_outer, double eps, const double* err, OctArgs& oa);
}  // namespace mpe

using namespace mpe;

namespace {

// 2^20 doubles (8 MiB): n_r * ceil(n_mm / 256) block partials
constexpr size_t kScratchDoubles = size_t(1) << 20;

// In host code this name is only a stand-in for the device array; its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with it current).
ewald_status_t scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(EWALD_ERR_HIP, "no current HIP device");
  if (dev < 0 || dev >= kMaxDevices) return set_error(EWALD_ERR_HIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return set_error(EWALD_ERR_HIP, "hipGetSymbolAddress of the scratch array failed");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return EWALD_OK;
}

}  // namespace

extern "C" ewald_status_t ewald_octupole_error_noalloc(const double box[3], int n_qm, const double* qm_xyz,
                                                       const double* omega, int n_mm, const double* mm_xyz,
                                                       const double* mm_q, int n_r, double r_first, double r_step,
                                                       double r_outer, double eps, double* err, double* r_cut,
                                                       void* stream) {
  clear_error();
  if (!box) return set_error(EWALD_ERR_ARG, "null box");
  OctArgs oa;
  ewald_status_t st = octupole_args(box, n_qm, qm_xyz, omega, n_mm, mm_xyz, mm_q, n_r, r_first, r_step, r_outer, eps,
                                    err, oa);
  if (st != EWALD_OK) return st;
  // partial sums: n_r candidates x one per 256 MM atoms (at least one slot each)
  const size_t blocks = n_mm > 0 ? ((size_t)n_mm + 255) / 256 : 1;
  if ((size_t)n_r * blocks > kScratchDoubles)
    return set_error(EWALD_ERR_CAPACITY,
                     "n_r * ceil(n_mm / 256) exceeds the 1048576 partial sums of the allocation-free scratch");
  double* part = nullptr;
  st = scratch_on_current_device(&part);
  if (st != EWALD_OK) return st;
  const hipError_t e = launch_octupole(oa, part, eps, err, r_cut, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(EWALD_ERR_HIP, hipGetErrorString(e));
  return EWALD_OK;
}
