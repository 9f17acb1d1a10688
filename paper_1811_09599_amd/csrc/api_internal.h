// Entry-point helpers shared between the C ABI's source files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

#include "../../include/qflex.h"

namespace qflex {

// Split-product workspace: two fp16 scale slots (padded), then the split A and B operands.
constexpr int64_t kSplitSlotBytes = 256;

inline int log2_exact(int64_t v) {  // log2 of a power of two, else -1
  if (v < 1) return -1;
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return (int64_t(1) << b) == v ? b : -1;
}

// Runs f, turning the library's errors into a status and the thread's last-error message.
qflex_status run_guarded(const std::function<void()>& f);

void gemm_split_c64_check(const void* A, const void* B, const void* C, int64_t M, int64_t N,
                          int64_t K, int32_t ta, int32_t tb, int64_t batch, int32_t precision);
void gemm_split_c64_run(const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K,
                        int32_t ta, int32_t tb, int64_t batch, int32_t precision, int32_t tile,
                        void* workspace, int64_t workspace_bytes, hipStream_t st);

}  // namespace qflex
