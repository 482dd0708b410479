// SSP-RK3 steps for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc): tdg_rk_step with its work
// buffer (the two intermediate stage states and, in the mixed modes, the three operand
// companions) taken from a fixed device array of this library instead of a caller buffer.
//
// The array is a file-scope __device__ variable, so every GPU the library runs on holds
// its own copy (kScratchBytes) from the moment the code object is loaded on that device
// until the process ends.  Host code never uses the variable's name as an address: the
// first call on a device, with that device current, looks up the copy's device address
// with hipGetSymbolAddress and keeps it per device; the stage kernels then receive that
// address like any caller work buffer.
//
// Every call on one GPU shares that GPU's array.  Nothing in it has to start at zero (the
// stages write each intermediate state and companion before reading it), but two calls
// that overlap in time on one GPU (different streams, threads or contexts) race on it:
// callers serialise them.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dg_launch.hpp"
#include "tetdg.h"

// 64 MiB: e.g. P3 FP64 up to ~25,000 elements, P1 FP64 up to ~200,000 (tdg_work_bytes).
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

extern "C" int tdg_rk_step_noalloc(tdg_ctx* c, void* U, double dt, int n_steps, void* hip_stream) {
  if (!c) return TDG_ERR_INVALID_ARG;
  size_t need = 0;
  if (tdg_work_bytes(c, &need) != TDG_OK) return tetdg::ctx_fail(c, TDG_ERR_STATE, "no mesh uploaded");
  if (need > kScratchBytes)
    return tetdg::ctx_fail(c, TDG_ERR_NOMEM,
                           "tdg_rk_step_noalloc: the work buffer of this mesh exceeds the library's 64 MiB "
                           "static scratch (see tdg_work_bytes); use tdg_rk_step with a caller buffer");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return tetdg::ctx_fail(c, TDG_ERR_HIP, "tdg_rk_step_noalloc: hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return tetdg::ctx_fail(c, TDG_ERR_UNSUPPORTED, "device index out of range");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return tetdg::ctx_fail(c, TDG_ERR_HIP, "tdg_rk_step_noalloc: hipGetSymbolAddress of the scratch failed");
      g_scratch_ptr[dev] = p;
    }
    ptr = g_scratch_ptr[dev];
  }
  return tdg_rk_step(c, U, ptr, dt, n_steps, hip_stream);
}
