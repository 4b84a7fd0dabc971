// A device scratch area that no call allocates: one file-scope array, which
// the HIP runtime places in every device's memory when it loads this code
// object and keeps there until the process ends.  The allocation-free
// decryption (pc2_decrypt_static) stages its CRT halves and window tables
// here.  Host code never passes the array's name to a kernel (on the host
// that name is only a stand-in for the symbol): it looks the device address
// up once per device, with that device current, and passes that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pc2.h"
#include "launch.hpp"

static_assert(PC2_STATIC_SCRATCH_BYTES % 256 == 0, "whole 256-byte blocks");

static __device__ __align__(256) uint32_t scratch[PC2_STATIC_SCRATCH_BYTES / 4];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
uint32_t* g_ptr[MAX_DEVICES] = {};
}  // namespace

namespace pc2k {

int static_scratch_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return 0;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return -1;
  uint32_t* ptr = nullptr;
  if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return -1;
  g_ptr[device] = ptr;
  return 0;
}

uint32_t* static_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace pc2k
