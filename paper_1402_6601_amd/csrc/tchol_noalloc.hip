// tchol_factor_solve_noalloc: the merged factor + solve launch with its
// scheduler scratch (header, dependency counters, task descriptors, successor
// lists, ticket list) in a fixed device array of this library instead of a
// caller workspace, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host the name
// stands for a host-side shadow, not device memory); it looks up the device
// address once per device with hipGetSymbolAddress and uses that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/tchol.h"

namespace tchol {
int64_t factor_solve_bytes(int64_t n, int64_t nb, int64_t nrhs, bool inv);
int32_t factor_solve_run(double* A, int64_t n, int64_t nb, double* B, int64_t nrhs, void* ws, int64_t ws_bytes,
                         void* stream, const tchol_opts* opts, bool pinned, bool inv);
}

static __device__ __align__(256) char scratch[TCHOL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on `dev` (the current device), looked up on
// the first call for that device.  Returns nullptr if the lookup failed.
void* scratch_ptr(int dev) {
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptr[dev] = p;
  }
  return ptr[dev];
}

}  // namespace

extern "C" {

int32_t tchol_factor_solve_noalloc(double* A, int64_t n, int64_t nb, double* B, int64_t nrhs, void* stream) {
  if (n < 0 || n > INT32_MAX) return -2;
  if (nb < TCHOL_NB_MIN || nb > TCHOL_NB_MAX || nb % 16 != 0) return -3;
  if (nrhs < 0 || nrhs > INT32_MAX) return -5;
  if (n == 0) return 0;
  if (!A) return -1;
  if (nrhs > 0 && !B) return -4;
  // the scheduler scratch this problem needs (host-side plan sizes only).  The
  // solve substitutes against the diagonal tiles: their explicit inverses
  // (n nb doubles) would not fit the fixed array at the orders it serves.
  const int64_t need = tchol::factor_solve_bytes(n, nb, nrhs, false);
  if (need < 0) return (int32_t)need;
  if (need > TCHOL_NOALLOC_SCRATCH_BYTES) return TCHOL_E_SCRATCH;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TCHOL_E_HIP;
  void* ws = scratch_ptr(dev);
  if (!ws) return TCHOL_E_HIP;
  return tchol::factor_solve_run(A, n, nb, B, nrhs, ws, TCHOL_NOALLOC_SCRATCH_BYTES, stream, nullptr, false, false);
}

}  // extern "C"
