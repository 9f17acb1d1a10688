// Fast frugal rejection sampling over open-qubit batches, and its sampling-error estimate.
#include "kernel_util.h"

#include <algorithm>

namespace qflex {
namespace dev {

// |a|^2 with each product and the sum rounded once: the accept decision below compares it
// with a threshold, so it must not depend on whether the compiler fuses a multiply-add.
__device__ inline double probability_rn(double2 a) {
#pragma clang fp contract(off)
  const double re2 = a.x * a.x;
  const double im2 = a.y * a.y;
  return re2 + im2;
}

// Wavefronts stride over the batches (paper, Methods, "Fast sampling technique": a batch is one
// closed-qubit bit-string with its open-qubit values).  Per batch, one round of loads brings
// the amplitudes (lane i: value i, 64 at a time), the visit order and the uniform numbers; the
// scaled probabilities x = N p go into the error estimate (sum of x > M, Methods, "Sampling from
// a non fully-thermalized Porter-Thomas distribution") and, for batches of at most 64 values,
// reach the visiting lanes by a shuffle instead of a second trip to memory.  Visits run 64 at
// a time: lane j takes visit r + j and accepts when u * M < x (probability min(1, N p / M));
// the batch keeps the earliest accepting visit (a ballot), so at most one value per batch.
// Wavefront w owns batches w, w + nw, ... and leaves its sum of the estimate in partial[w].
__global__ void __launch_bounds__(256) frugal_sample_kernel(
    const double2* __restrict__ amps, int64_t n_batch, int64_t batch_len,
    const int32_t* __restrict__ order, const double* __restrict__ u, int32_t n_c, double dim,
    double m, int32_t* __restrict__ accepted, double* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4, w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= n_batch) return;  // whole wavefronts leave together
  double tw = 0.0;  // this lane's share of the estimate over the wavefront's batches
  for (int64_t b = w; b < n_batch; b += nw) {
    const double2* a = amps + b * batch_len;
    const int32_t* ob = order + b * n_c;
    const double* ub = u + b * n_c;
    // the first round of visits is loaded with the amplitudes
    int32_t s = 0;
    double uj = 0.0;
    if (lane < n_c) s = ob[lane], uj = ub[lane];
    double x0 = 0.0;
    for (int64_t i = lane; i < batch_len; i += 64) {
      const double x = dim * probability_rn(a[i]);
      if (i < 64) x0 = x;
      if (x > m) tw += x;
    }
    int32_t pick = -1;
    for (int32_t r = 0; r < n_c; r += 64) {
      const int32_t j = r + lane;
      if (r > 0 && j < n_c) s = ob[j], uj = ub[j];
      const bool bad = j < n_c && (s < 0 || (int64_t)s >= batch_len);
      if (__ballot(bad)) {
        pick = -2;
        break;
      }
      double x;
      if (batch_len <= 64) {
        x = __shfl(x0, s & 63, 64);
      } else {
        x = j < n_c ? dim * probability_rn(a[s]) : 0.0;
      }
      const uint64_t hit = __ballot(j < n_c && uj * m < x);
      if (hit) {
        pick = __shfl(s, __builtin_ctzll(hit), 64);
        break;
      }
    }
    if (lane == 0) accepted[b] = pick;
  }
  tw = wave_sum(tw);
  if (lane == 0) partial[w] = tw;
}

// tail = (sum of partial[0 .. n)) / count, by one workgroup in a fixed order
__global__ void __launch_bounds__(256) tail_sum_kernel(const double* __restrict__ partial,
                                                       int64_t n, double count,
                                                       double* __restrict__ tail) {
  __shared__ double part[4];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) t += partial[i];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) *tail = ((part[0] + part[1]) + (part[2] + part[3])) / count;
}

void frugal_sample(const double2* amps, int64_t n_batch, int64_t batch_len, const int32_t* order,
                   const double* u, int32_t n_c, int32_t n_qubits, double m, int32_t* accepted,
                   double* partial, double* tail, hipStream_t s) {
  if (n_batch <= 0) return;
  const double dim = ldexp(1.0, n_qubits);
  // enough wavefronts to fill the device (8 workgroups of 4 per compute unit), each walking
  // many batches
  const int64_t blocks = std::min<int64_t>((n_batch + 3) / 4, 256 * 8);
  hipLaunchKernelGGL(frugal_sample_kernel, dim3((unsigned)blocks), dim3(256), 0, s, amps, n_batch,
                     batch_len, order, u, n_c, dim, m, accepted, partial);
  check_launch("frugal_sample");
  hipLaunchKernelGGL(tail_sum_kernel, dim3(1), dim3(256), 0, s, partial,
                     std::min<int64_t>(blocks * 4, n_batch), (double)n_batch * (double)batch_len,
                     tail);
  check_launch("tail_sum");
}

}  // namespace dev
}  // namespace qflex
