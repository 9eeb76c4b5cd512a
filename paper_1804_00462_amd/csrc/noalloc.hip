// sorsvd() for callers that cannot allocate device memory (code under HIP
// graph capture, serving loops, harnesses that forbid hipMalloc): the
// workspace is a fixed array of this library in device memory, of
// SORSVD_NOALLOC_BYTES, one per device that calls it (held until the process
// ends). Every call on a device uses that device's array and leaves its
// contents behind; the sequence of sorsvd() writes every workspace word it
// reads first, so nothing needs clearing between calls. Calls that overlap
// on one device (on different streams or threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sorsvd.h"

namespace {

static __device__ __align__(256) unsigned char scratch[SORSVD_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device (null: not taken yet)

// The array's address on the current device, taken once per device with that
// device current (the name `scratch` is a host-side stand-in, not a device
// address).
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SORSVD_EHIP;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SORSVD_EHIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SORSVD_OK;
}

}  // namespace

extern "C" int sorsvd_noalloc(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, int64_t k,
                              int32_t q, uint64_t seed, void* U, int64_t ldu, double* S, void* V, int64_t ldv,
                              void* stream, const sorsvd_opts* opts, sorsvd_info* info) {
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc != SORSVD_OK) return rc;
  // argument checks and the workspace bound (SORSVD_EWORKSPACE beyond the
  // array) are sorsvd()'s, before anything is enqueued
  rc = sorsvd(A, lda, a_type, m, n, k, q, seed, U, ldu, S, V, ldv, ws, SORSVD_NOALLOC_BYTES, stream, opts);
  if (rc == SORSVD_OK && info) rc = sorsvd_read_info(ws, info, stream);
  return rc;
}
