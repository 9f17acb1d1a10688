// The split-precision complex product on a library-owned device buffer: for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  The buffer is a static device array, so each GPU the library runs on
// holds its own copy from the moment the code object is loaded until the process ends.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/qflex_kernels.h"
#include "api_internal.h"
#include "grid.h"

// The staging buffer of qflex_gemm_split_c64_noalloc: fp16 scale slots, then the split
// operands.  In host code `scratch` is only a stand-in for the symbol, not a device address:
// every host use goes through the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[QFLEX_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up on the first call on
// that device (with that device current) and kept.
void* scratch_for_current_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    qflex::fail(QFLEX_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) qflex::fail(QFLEX_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      qflex::fail(QFLEX_E_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" qflex_status qflex_gemm_split_c64_noalloc(const void* A, const void* B, void* C,
                                                     int64_t M, int64_t N, int64_t K,
                                                     int32_t ta, int32_t tb, int64_t batch,
                                                     int32_t precision, void* stream) {
  return qflex::run_guarded([&] {
    qflex::gemm_split_c64_check(A, B, C, M, N, K, ta, tb, batch, precision);
    const int64_t need = qflex_gemm_split_workspace(M, N, K, batch);
    if (need > QFLEX_NOALLOC_SCRATCH_BYTES)
      qflex::fail(QFLEX_E_INVALID,
                  "the split operands need " + std::to_string(need) +
                      " bytes of scratch, more than the library's " +
                      std::to_string((long long)QFLEX_NOALLOC_SCRATCH_BYTES) +
                      "; use qflex_gemm_split_c64 with a workspace");
    qflex::gemm_split_c64_run(A, B, C, M, N, K, ta, tb, batch, precision, -1,
                              scratch_for_current_device(), QFLEX_NOALLOC_SCRATCH_BYTES,
                              static_cast<hipStream_t>(stream));
  });
}
