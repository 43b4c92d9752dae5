// tc_ttc_solve_noalloc: tc_ttc_solve for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The fused pass's partial sums go to a scratch array of
// fixed size that lives in this library's device memory; nothing is allocated
// or freed, here or in the kernels it launches.
//
// The array is a file-scope __device__ variable, so each GPU holds its own copy
// at its own address.  In host code its name is only a host-side stand-in:
// the device address is taken once per device with hipGetSymbolAddress (with
// that device current) and kept; only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = TC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// The current device's address of `scratch`, looked up on first use.
int scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TC_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return TC_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TC_OK;
}

}  // namespace

extern "C" int tc_ttc_solve_noalloc(const tc_tensor* prev, const tc_tensor* next, int32_t levels,
                                    tc_ttc_level* levels_out, tc_ttc_pick* pick_out, void* stream) {
  if (!prev || !next || !levels_out || !pick_out) return TC_EINVAL;
  // the size check first: a pair whose partial sums exceed the array is
  // refused before anything is looked up or launched
  size_t need = 0;
  if (prev->ndim != 2) return TC_ESHAPE;
  int st = tc_ttc_workspace_size(prev->shape[0], prev->shape[1], levels, &need);
  if (st != TC_OK) return st;
  if (need > kScratchBytes) return TC_ENOMEM;
  void* ws = nullptr;
  if ((st = scratch_for_current_device(&ws)) != TC_OK) return st;
  // every partial the finishing pass reads is written by the fused pass of
  // the same call, so no part of the array has to start at zero
  return tc_ttc_solve(prev, next, levels, ws, kScratchBytes, levels_out, pick_out, stream);
}
