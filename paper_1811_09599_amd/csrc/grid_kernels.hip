// Time collapse of every qubit's gates into one tensor per qubit, and its adjoint.
#include "kernel_util.h"

namespace qflex {
namespace dev {
// =============================================================================================
// Grid build: time collapse of every qubit's gates (paper, Methods B.1).
// One thread per (qubit, value of the qubit's link bonds): it carries the 2-vector
// |v> = P_t(k_t) ... P_1(k_1) |0> in FP64 through the qubit's pieces, each piece's matrix picked
// by that piece's bond digits, and stores <0|v>, <1|v> as complex64 at the addresses the
// plan's layout assigns to (output bit, bond values).
// =============================================================================================
__global__ void __launch_bounds__(256) grid_build_kernel(const GridQubit* __restrict__ qd,
                                                         const GridPiece* __restrict__ pieces,
                                                         const double2* __restrict__ mats,
                                                         const int32_t* __restrict__ pos,
                                                         float2* __restrict__ out) {
  const GridQubit d = qd[blockIdx.y];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t(1) << d.nlb)) return;
  double2 v0 = make_double2(1.0, 0.0), v1 = make_double2(0.0, 0.0);
  for (int p = d.piece_begin; p < d.piece_end; ++p) {
    const GridPiece pc = pieces[p];
    const int k = (int)((c >> pc.kshift) & pc.kmask);
    const double2* M = mats + 4 * (pc.mat + k);
    const double2 a = cmul(M[0], v0), b = cmul(M[1], v1);
    const double2 e = cmul(M[2], v0), f = cmul(M[3], v1);
    v0 = make_double2(a.x + b.x, a.y + b.y);
    v1 = make_double2(e.x + f.x, e.y + f.y);
  }
  int64_t addr = 0;
  for (int j = 0; j < d.nlb; ++j) addr |= ((c >> (d.nlb - 1 - j)) & 1) << pos[d.pos_base + j];
  out[d.offset + addr] = make_float2((float)v0.x, (float)v0.y);
  out[d.offset + (addr | (int64_t(1) << d.pos_out))] = make_float2((float)v1.x, (float)v1.y);
}

void grid_build(const GridQubit* q, int n_qubits, int max_nlb, const GridPiece* pieces,
                const double2* mats, const int32_t* pos, float2* out, hipStream_t s) {
  const int64_t combos = int64_t(1) << max_nlb;
  dim3 grid((unsigned)((combos + 255) / 256), (unsigned)n_qubits);
  hipLaunchKernelGGL(grid_build_kernel, grid, dim3(256), 0, s, q, pieces, mats, pos, out);
  check_launch("grid_build");
}

// =============================================================================================
// Adjoint of the contraction (gradients).
// =============================================================================================

// One thread per (qubit, bond values): recompute the kets v_t = P_t ... P_1 |0> of the qubit's
// time line (kept in private memory), then carry the cotangent row vector
// u_L = (tbar[o=0], tbar[o=1]) backwards: dP_t[a][b] += u_t[a] v_{t-1}[b], u_{t-1} = u_t P_t.
// Contributions to each piece matrix are summed over the wavefront, then added atomically.
__global__ void __launch_bounds__(256) grid_adjoint_kernel(const GridQubit* __restrict__ qd,
                                                           const GridPiece* __restrict__ pieces,
                                                           const double2* __restrict__ mats,
                                                           const int32_t* __restrict__ pos,
                                                           const double2* __restrict__ tbar,
                                                           double2* __restrict__ pbar) {
  const GridQubit d = qd[blockIdx.y];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = c < (int64_t(1) << d.nlb);
  if ((int64_t)blockIdx.x * blockDim.x >= (int64_t(1) << d.nlb)) return;  // whole block idle
  const int np = d.piece_end - d.piece_begin;
  double2 v0[kMaxPiecesGrad + 1], v1[kMaxPiecesGrad + 1];
  v0[0] = make_double2(1.0, 0.0);
  v1[0] = make_double2(0.0, 0.0);
  for (int t = 0; t < np; ++t) {
    const GridPiece pc = pieces[d.piece_begin + t];
    const int k = active ? (int)((c >> pc.kshift) & pc.kmask) : 0;
    const double2* M = mats + 4 * (pc.mat + k);
    v0[t + 1] = cadd(cmul(M[0], v0[t]), cmul(M[1], v1[t]));
    v1[t + 1] = cadd(cmul(M[2], v0[t]), cmul(M[3], v1[t]));
  }
  double2 u0 = make_double2(0, 0), u1 = make_double2(0, 0);
  if (active) {
    int64_t addr = 0;
    for (int j = 0; j < d.nlb; ++j) addr |= ((c >> (d.nlb - 1 - j)) & 1) << pos[d.pos_base + j];
    u0 = tbar[d.offset + addr];
    u1 = tbar[d.offset + (addr | (int64_t(1) << d.pos_out))];
  }
  const int lane = threadIdx.x & 63;
  for (int t = np - 1; t >= 0; --t) {
    const GridPiece pc = pieces[d.piece_begin + t];
    const int k = active ? (int)((c >> pc.kshift) & pc.kmask) : 0;
    const double2 a0 = v0[t], a1 = v1[t];
    // outer product u (row) x v_{t-1} (column)
    const double2 g[4] = {cmul(u0, a0), cmul(u0, a1), cmul(u1, a0), cmul(u1, a1)};
    for (int kk = 0; kk <= pc.kmask; ++kk) {
      const bool mine = active && k == kk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double re = wave_sum(mine ? g[e].x : 0.0);
        const double im = wave_sum(mine ? g[e].y : 0.0);
        if (lane == 0 && (re != 0.0 || im != 0.0)) {
          atomicAdd(&pbar[4 * (pc.mat + kk) + e].x, re);
          atomicAdd(&pbar[4 * (pc.mat + kk) + e].y, im);
        }
      }
    }
    const double2* M = mats + 4 * (pc.mat + k);
    const double2 n0 = cadd(cmul(u0, M[0]), cmul(u1, M[2]));
    const double2 n1 = cadd(cmul(u0, M[1]), cmul(u1, M[3]));
    u0 = n0;
    u1 = n1;
  }
}

void grid_adjoint(const GridQubit* q, int n_qubits, int max_nlb, const GridPiece* pieces,
                  const double2* mats, const int32_t* pos, const double2* tbar, double2* pbar,
                  hipStream_t s) {
  const int64_t combos = int64_t(1) << max_nlb;
  dim3 grid((unsigned)((combos + 255) / 256), (unsigned)n_qubits);
  hipLaunchKernelGGL(grid_adjoint_kernel, grid, dim3(256), 0, s, q, pieces, mats, pos, tbar, pbar);
  check_launch("grid_adjoint");
}
}  // namespace dev
}  // namespace qflex
