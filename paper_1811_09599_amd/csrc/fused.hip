// The fused small-plan contraction (see fused_contract in kernels.h).
#include "kernel_util.h"

namespace qflex {
namespace dev {

namespace {

struct FusedArgs {
  FusedPlan p;
  const float2* grid;
  const int64_t* offs;
  int64_t nbs, b0;
  double2* acc;
  int32_t overwrite;  // 1: the first slice writes the amplitudes instead of adding to them
  int32_t nslices;
  int64_t slices[kFusedMaxSlices];
};

__global__ void __launch_bounds__(kFusedThreads) fused_contract_kernel(const FusedArgs a) {
  extern __shared__ __attribute__((aligned(16))) float2 lds[];
  __shared__ int32_t digit[kFusedMaxCuts];
  __shared__ uint32_t changed_s;
  __shared__ int64_t boff[kFusedMaxQubits];  // this bit-string's offset of each qubit tensor
  static_assert(sizeof(FusedStep) == 32, "step descriptors of 32 bytes");
  const int tid = threadIdx.x;
  const int64_t bs = a.b0 + blockIdx.x;  // the bit-string, within the circuit's
  const FusedPlan& p = a.p;
  // the step descriptors and index tables, copied once after the tensor image
  FusedStep* steps = reinterpret_cast<FusedStep*>(lds + p.lds_elems);
  uint16_t* tabs = reinterpret_cast<uint16_t*>(steps + p.nsteps);
  {
    const int32_t words = p.nsteps * (int32_t)(sizeof(FusedStep) / 4);
    const int32_t* src = reinterpret_cast<const int32_t*>(p.steps);
    int32_t* dst = reinterpret_cast<int32_t*>(steps);
    for (int32_t i = tid; i < words; i += kFusedThreads) dst[i] = src[i];
    for (int32_t i = tid; i < p.ntab; i += kFusedThreads) tabs[i] = p.tables[i];
    // the offsets table may live in host memory: each entry is read once (the first slice's
    // barrier orders these writes before their use)
    for (int32_t q = tid; q < p.nq; q += kFusedThreads) {
      const int32_t row = p.qubits[q].out_row;
      boff[q] = row >= 0 ? a.offs[row * a.nbs + bs] : 0;
    }
  }
  for (int si = 0; si < a.nslices; ++si) {
    // cut values of the slice (the last cut least significant) and the cuts that changed
    if (tid == 0) {
      int64_t rem = a.slices[si];
      uint32_t changed = 0;
      for (int c = p.ncut - 1; c >= 0; --c) {
        const int32_t d = (int32_t)(rem & ((int64_t(1) << p.cut_bits[c]) - 1));
        rem >>= p.cut_bits[c];
        if (si == 0 || d != digit[c]) changed |= 1u << c;
        digit[c] = d;
      }
      changed_s = changed;
    }
    __syncthreads();
    const uint32_t changed = changed_s;
    const bool fresh = si == 0;
    // the qubit tensors' free parts for this bit-string and slice: the loads of 8 tensors
    // are issued before any of them is stored, so that their latencies overlap
    constexpr int QB = 8;
    for (int q0 = 0; q0 < p.nq; q0 += QB) {
      float2 v[QB][2];
      int64_t off[QB];
      int32_t n[QB];
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        const int q = q0 + j;
        n[j] = 0;
        off[j] = 0;
        if (q < p.nq) {
          const FusedQubit& Q = p.qubits[q];
          if (fresh || (Q.deps & changed)) {
            int64_t o = Q.grid_off;
            for (int c = 0; c < Q.ncut; ++c) o += (int64_t)digit[Q.cut[c]] << Q.shift[c];
            o += boff[q];
            off[j] = o;
            n[j] = 1 << Q.free_bits;
          }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int32_t i = tid + t * kFusedThreads;
          if (i < n[j]) v[j][t] = a.grid[off[j] + i];
        }
      }
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        if (n[j] == 0) continue;
        const int32_t base = p.qubits[q0 + j].lds;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int32_t i = tid + t * kFusedThreads;
          if (i < n[j]) lds[base + i] = v[j][t];
        }
        // tensors larger than two elements per thread
        for (int32_t i = tid + 2 * kFusedThreads; i < n[j]; i += kFusedThreads)
          lds[base + i] = a.grid[off[j] + i];
      }
    }
    __syncthreads();
    for (int k = 0; k < p.nsteps; ++k) {
      const FusedStep& S = steps[k];
      if (!fresh && !(S.deps & changed)) continue;
      const int32_t K = 1 << S.kb, N = 1 << S.nb, MN = 1 << (S.mb + S.nb);
      const uint16_t* xm = tabs + S.tab;
      const uint16_t* yn = xm + (1 << S.mb);
      const uint16_t* kx = yn + N;
      const uint16_t* ky = kx + K;
      const float2* X = lds + S.x;
      const float2* Y = lds + S.y;
      for (int32_t i = tid; i < MN; i += kFusedThreads) {
        const int32_t xo = xm[i >> S.nb];
        const int32_t yo = yn[i & (N - 1)];
        float re = 0.f, im = 0.f;
        int32_t kk = 0;
        // four k at a time, so that their LDS reads are in flight together
        for (; kk + 4 <= K; kk += 4) {
          float2 u[4], v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            u[j] = X[xo + kx[kk + j]];
            v[j] = Y[ky[kk + j] + yo];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            re = fmaf(u[j].x, v[j].x, re);
            re = fmaf(-u[j].y, v[j].y, re);
            im = fmaf(u[j].x, v[j].y, im);
            im = fmaf(u[j].y, v[j].x, im);
          }
        }
        for (; kk < K; ++kk) {
          const float2 u = X[xo + kx[kk]], v = Y[ky[kk] + yo];
          re = fmaf(u.x, v.x, re);
          re = fmaf(-u.y, v.y, re);
          im = fmaf(u.x, v.y, im);
          im = fmaf(u.y, v.x, im);
        }
        lds[S.out + i] = make_float2(re, im);
      }
      __syncthreads();
    }
    // the slice's result, added in FP64 (one workgroup per bit-string: no other writer)
    for (int32_t e = tid; e < p.namp; e += kFusedThreads) {
      const float2 r = lds[p.result + e];
      double2& d = a.acc[bs * p.namp + p.bidx[e]];
      if (si == 0 && a.overwrite) {
        d = make_double2((double)r.x, (double)r.y);
      } else {
        d.x += (double)r.x;
        d.y += (double)r.y;
      }
    }
    __syncthreads();
  }
}

}  // namespace

void fused_setup() {
  // dynamic LDS beyond the default limit, up to the largest plan image
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_contract_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(sizeof(float2) * kFusedMaxLdsElems));
  if (e != hipSuccess) throw std::runtime_error(std::string("fused_setup: ") + hipGetErrorString(e));
}

void fused_contract(const FusedPlan& p, const float2* grid, const int64_t* offs, int64_t nbs,
                    int64_t b0, int64_t nb, const int64_t* slices, int nslices, double2* acc,
                    bool overwrite, hipStream_t s) {
  if (nb < 1 || nslices < 1) return;
  if (p.lds_elems < 1 || p.lds_elems > kFusedMaxLdsElems || p.nsteps > kFusedMaxSteps ||
      p.nq > kFusedMaxQubits || p.ncut > kFusedMaxCuts || b0 < 0 || b0 + nb > nbs)
    throw std::runtime_error("fused_contract: plan outside the kernel's limits");
  const size_t bytes = sizeof(float2) * (size_t)p.lds_elems + sizeof(FusedStep) * p.nsteps +
                       sizeof(uint16_t) * (size_t)p.ntab;
  if (bytes > sizeof(float2) * kFusedMaxLdsElems)
    throw std::runtime_error("fused_contract: plan image too large for LDS");
  FusedArgs a;
  a.p = p;
  a.grid = grid;
  a.offs = offs;
  a.nbs = nbs;
  a.acc = acc;
  for (int s0 = 0; s0 < nslices; s0 += kFusedMaxSlices) {
    a.overwrite = overwrite && s0 == 0;
    a.nslices = std::min(kFusedMaxSlices, nslices - s0);
    for (int i = 0; i < a.nslices; ++i) a.slices[i] = slices[s0 + i];
    for (int64_t c0 = 0; c0 < nb; c0 += 65535) {
      a.b0 = b0 + c0;
      const unsigned grid_x = (unsigned)std::min<int64_t>(65535, nb - c0);
      hipLaunchKernelGGL(fused_contract_kernel, dim3(grid_x), dim3(kFusedThreads), bytes, s, a);
      check_launch("fused_contract");
    }
  }
}

}  // namespace dev
}  // namespace qflex
