// fmm_invariants_noalloc: the invariant reductions of fmm_invariants for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops).  The per-block partial sums live in a file-scope
// device array instead of a context's workspace, and a second kernel adds
// them in block order on the device, so nothing is allocated, copied to the
// host or waited for.
//
// Host code never passes `scratch` itself to a kernel: in host code that name
// is a host-side stand-in, not a device address.  Its device address is looked
// up once per device with hipGetSymbolAddress (every GPU holds its own copy)
// and that pointer is what the kernels receive.
#include <mutex>

#include "../../include/fmm355.h"
#include "common.h"
#include "hhs_kernels.h"

namespace {

constexpr int kScratchDoubles = FMM_INV_BLOCKS * 12;  // 48 KiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices];  // device address of `scratch`, per device (null until looked up)

// out[k] = sum over blocks b = 0, 1, ... of part[b * 12 + k], added in that
// order in FP64: the order in which fmm_invariants adds them on the host.
__global__ void k_invariants_final(const double *__restrict__ part, int nblk,
                                   double *__restrict__ out) {
  const int k = threadIdx.x;
  if (k >= 12) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[b * 12 + k];
  out[k] = s;
}

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
fmm_status scratch_ptr(double **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FMM_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FMM_EDEVICE;
    g_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_ptr[dev];
  return FMM_OK;
}

}  // namespace

extern "C" fmm_status fmm_invariants_noalloc(void *stream, const double *pos, const double *vel,
                                             const double *mass, const double *acc,
                                             const double *pot, int64_t n, double *out) {
  if (!out || n < 0) return FMM_EINVAL;
  double *part = nullptr;
  const fmm_status st = scratch_ptr(&part);
  if (st != FMM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_invariants(pos, vel, mass, acc, pot, n, part, FMM_INV_BLOCKS, s);
  hipLaunchKernelGGL(k_invariants_final, dim3(1), dim3(64), 0, s, part, FMM_INV_BLOCKS, out);
  return hipGetLastError() == hipSuccess ? FMM_OK : FMM_EDEVICE;
}
