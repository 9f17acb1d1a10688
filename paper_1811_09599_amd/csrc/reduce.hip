// FP64 reductions: slice accumulation, zero fill, cotangent seeds.
#include "kernel_util.h"

namespace qflex {
namespace dev {

// =============================================================================================
// FP64 accumulation of a slice's result into the amplitude batch (paper, Methods B.1: the
// amplitude is the sum of the path contributions; Methods C.1: a fraction of them).
// =============================================================================================
__global__ void accumulate_kernel(const float2* __restrict__ res, const int64_t* __restrict__ r_off,
                                  int64_t r_bs, int64_t r_add, int64_t n,
                                  const uint32_t* __restrict__ bidx, double2* __restrict__ amps,
                                  int64_t amp_stride) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int b = blockIdx.y;
  const float2 v = res[r_add + (r_off ? r_off[b] : b * r_bs) + e];
  double2* a = amps + b * amp_stride + bidx[e];
  double2 t = *a;
  t.x += (double)v.x;
  t.y += (double)v.y;
  *a = t;
}

void accumulate(const float2* res, const int64_t* r_off, int64_t r_bs, int64_t r_add, int64_t n,
                const uint32_t* bidx, double2* amps, int64_t amp_stride, int batch,
                hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)batch);
  hipLaunchKernelGGL(accumulate_kernel, grid, dim3(256), 0, s, res, r_off, r_bs, r_add, n, bidx,
                     amps, amp_stride);
  check_launch("accumulate");
}

__global__ void fill_zero_kernel(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

void fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  check_launch("fill_zero");
}
__global__ void seed_cotangent_kernel(const double2* __restrict__ gbar,
                                      const uint32_t* __restrict__ bidx, int64_t n, int64_t namp,
                                      float2* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int b = blockIdx.y;
  const double2 v = gbar[(int64_t)b * namp + bidx[e]];
  dst[(int64_t)b * n + e] = make_float2((float)v.x, (float)-v.y);
}

void seed_cotangent(const double2* gbar, const uint32_t* bidx, int64_t n, int64_t namp,
                    int batch, float2* dst, hipStream_t s) {
  hipLaunchKernelGGL(seed_cotangent_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)batch),
                     dim3(256), 0, s, gbar, bidx, n, namp, dst);
  check_launch("seed_cotangent");
}

__global__ void xeb_cotangent_kernel(const double2* __restrict__ amps, int64_t n, double scale,
                                     double2* __restrict__ gbar, double* __restrict__ sum_sq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double2 a = amps[i];
    gbar[i] = make_double2(scale * a.x, scale * a.y);
    v = a.x * a.x + a.y * a.y;
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(sum_sq, v);
}

void xeb_cotangent(const double2* amps, int64_t n, double scale, double2* gbar, double* sum_sq,
                   hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(xeb_cotangent_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     amps, n, scale, gbar, sum_sq);
  check_launch("xeb_cotangent");
}
}  // namespace dev
}  // namespace qflex
