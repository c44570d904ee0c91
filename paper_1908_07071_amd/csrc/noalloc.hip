// lor_apply_P_noalloc: the preconditioner application z = B r of eq. as
// (eq. dg-as for DG) for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The scratch vectors of B -- the coarse-space residual and correction
// (n_c values each) and, for DG, the conforming residual and correction of
// E B E^T (one L-vector each) -- live in one file-scope device array instead
// of the handle's workspace.  Every GPU the library runs on holds its own
// copy of the array until the process ends; the device address of that copy
// is looked up once per device (hipGetSymbolAddress, at lor_setup on the
// device current there) and only that address is handed to kernels: in host
// code the array's name is a host-side stand-in, not a device pointer.
//
// All calls on one GPU share the array, so two calls that overlap on one GPU
// (different streams or threads) race.  Nothing in it must start at zero:
// every scratch vector is written completely before it is read.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lor_handle.h"

namespace {

constexpr size_t kScratchDoubles = size_t(1) << 20;  // 8 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

int noalloc_register_device(int device) {
  if (device < 0 || device >= kMaxDevices) return LOR_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return LOR_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return LOR_EHIP;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LOR_EHIP;
  g_ptr[device] = static_cast<double *>(p);
  return LOR_OK;
}

extern "C" int lor_apply_P_noalloc(lor_handle_t *h, const double *r_dev, double *z_dev,
                                   void *stream) {
  if (!h || !r_dev || !z_dev || r_dev == z_dev) return LOR_EINVAL;
  if (!h->has_prec) return LOR_ESTATE;
  if (h->nn && h->nn_mode != LOR_NN_OFF) return LOR_ESTATE;  // the network path is not covered
  if (h->device < 0 || h->device >= kMaxDevices) return LOR_EINVAL;
  double *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ptr = g_ptr[h->device];
  }
  if (!ptr) return LOR_ESTATE;  // registered by lor_setup on this device
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return LOR_EHIP;
  if (cur != h->device) return LOR_EINVAL;  // the handle's device must be current
  return apply_P_scratch(h, ptr, kScratchDoubles, r_dev, z_dev, static_cast<hipStream_t>(stream));
}

extern "C" int lor_noalloc_scratch_bytes(const lor_handle_t *h, size_t *needed, size_t *capacity) {
  if (!h || !needed || !capacity) return LOR_EINVAL;
  *needed = apply_P_scratch_doubles(h) * sizeof(double);
  *capacity = kScratchDoubles * sizeof(double);
  return LOR_OK;
}
