// XMS rotation for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops): the same kernels as xms_rotate, with
// the one intermediate -- the Fock operator in the reference space, F^ref of
// Eq. 3 -- in a fixed file-scope device array instead of a buffer allocated
// per call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/caspt2.h"
#include "kernels.hpp"

using namespace caspt2;

// F^ref of at most XMS_NOALLOC_MAX_STATES states (2 KiB).  Each GPU holds its
// own copy until the process ends; every call on a GPU shares it.
constexpr int XMS_NOALLOC_MAX_STATES = 16;
constexpr int XMS_NOALLOC_SCRATCH = XMS_NOALLOC_MAX_STATES * XMS_NOALLOC_MAX_STATES;
static __device__ __align__(256) double scratch[XMS_NOALLOC_SCRATCH];

namespace {

// device address of the array per device, looked up once per device with
// that device current (the array's name is a host-side stand-in)
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;

hipError_t scratch_of_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int xms_rotate_noalloc(int32_t nact, int32_t nst, const double* f_act, const double* rdm1, double* U, double* e0,
                       void* stream) {
  if (nact < 0 || nst <= 0 || (nact > 0 && (!f_act || !rdm1)) || !U || !e0) return CASPT2_E_ARG;
  if (nst > XMS_NOALLOC_MAX_STATES) return CASPT2_E_ARG;
  double* F = nullptr;
  if (scratch_of_current_device(&F) != hipSuccess) return CASPT2_E_DEVICE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // F is written whole by the first kernel: nothing to clear
  if (xms_fref(nact, nst, f_act, rdm1, F, s) != hipSuccess) return CASPT2_E_DEVICE;
  if (small_eigh(nst, F, e0, U, s) != hipSuccess) return CASPT2_E_DEVICE;
  return CASPT2_OK;
}

}  // extern "C"
