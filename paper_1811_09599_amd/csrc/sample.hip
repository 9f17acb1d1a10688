// Fast frugal rejection sampling over open-qubit batches, and its sampling-error estimate.
#include "kernel_util.h"

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

// One wavefront per batch (paper, Methods, "Fast sampling technique": one closed-qubit
// bit-string with its open-qubit values).  Visits run 64 at a time: lane j of a round takes
// visit r + j, accepts when u * M < N p (probability min(1, N p / M)), and the batch keeps
// the earliest accepting visit (a ballot), so at most one bit-string per batch.  The same
// wavefront sums N p over the batch's amplitudes with N p > M (Methods, "Sampling from a non
// fully-thermalized Porter-Thomas distribution") into partial[b], in a fixed order.
__global__ void __launch_bounds__(256) frugal_sample_kernel(
    const double2* __restrict__ amps, int64_t n_batch, int64_t batch_len,
    const int32_t* __restrict__ order, const double* __restrict__ u, int32_t n_c, double dim,
    double m, int32_t* __restrict__ accepted, double* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= n_batch) return;  // whole wavefronts leave together
  const double2* a = amps + b * batch_len;
  int32_t pick = -1;
  for (int32_t r = 0; r < n_c; r += 64) {
    const int32_t j = r + lane;
    bool bad = false, acc = false;
    int32_t s = 0;
    if (j < n_c) {
      s = order[b * n_c + j];
      bad = s < 0 || (int64_t)s >= batch_len;
      if (!bad) acc = u[b * n_c + j] * m < dim * probability_rn(a[s]);
    }
    if (__ballot(bad)) {
      pick = -2;
      break;
    }
    const uint64_t hit = __ballot(acc);
    if (hit) {
      pick = __shfl(s, __builtin_ctzll(hit), 64);
      break;
    }
  }
  double t = 0.0;
  for (int64_t i = lane; i < batch_len; i += 64) {
    const double x = dim * probability_rn(a[i]);
    if (x > m) t += x;
  }
  t = wave_sum(t);
  if (lane == 0) {
    accepted[b] = pick;
    partial[b] = t;
  }
}

// tail = (sum over b of partial[b]) / count, by one workgroup in a fixed order
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
  hipLaunchKernelGGL(frugal_sample_kernel, dim3((unsigned)((n_batch + 3) / 4)), dim3(256), 0, s,
                     amps, n_batch, batch_len, order, u, n_c, dim, m, accepted, partial);
  check_launch("frugal_sample");
  hipLaunchKernelGGL(tail_sum_kernel, dim3(1), dim3(256), 0, s, partial, n_batch,
                     (double)n_batch * (double)batch_len, tail);
  check_launch("tail_sum");
}

}  // namespace dev
}  // namespace qflex
