// Adjoint contraction: gradients of a real loss of the amplitudes with respect to gate
// entries and fSim angles.
//
// The paper computes amplitudes only; this is the reverse-mode counterpart of the same plan.
// With W = conj(dL/d conj psi) per amplitude (holomorphic seed), every step Z = X Y of the
// forward plan is reversed as Xbar = Zbar Y^T and Ybar = X^T Zbar (plain transposes: the
// contraction is holomorphic in its tensors) followed by the inverse permutation.  For each
// batch of bit-strings and each selected slice, the forward pass keeps only the slice's
// checkpoints (the intermediates one segment of consecutive steps hands to a later one, see
// make_grad_layout) and its last segment; the reverse sweep takes the segments from the last,
// recomputing each earlier one from its checkpoints and the qubit tensors before reversing it.
// The qubit-tensor cotangents are summed in FP64.  The time collapse is then reversed per qubit
// (the per-piece kets are recomputed, not stored), giving the cotangent of every 2x2 piece
// matrix, and the host maps pieces back to gate entries: dL/dtheta = 2 Re sum_e Gbar[e]
// dG[e]/dtheta.  In graph mode a call with one slice per circuit replays the launches the
// previous such call captured (same shapes, slices and buffers).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "grid.h"

namespace qflex {

#define QHIPG(expr)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      fail(e_ == hipErrorOutOfMemory ? QFLEX_E_NOMEM : QFLEX_E_DEVICE,                      \
           std::string(#expr) + ": " + hipGetErrorString(e_));                              \
  } while (0)

namespace {

struct GView {
  const float2* base = nullptr;
  const int64_t* off = nullptr;
  int64_t bs = 0, add = 0;
};

std::vector<int> cat(std::vector<int> a, const std::vector<int>& b) {
  a.insert(a.end(), b.begin(), b.end());
  return a;
}

}  // namespace

void contract_grad(qflex_grid* g, const uint8_t* bits, const int64_t* bs_offsets,
                   double fidelity, uint64_t seed, const int64_t* slice_ids,
                   const int64_t* slice_offsets, const double* cot, int32_t cot_on_device,
                   double* amps_out, double* grad_gates, double* grad_params, double* loss,
                   bool out_on_device, hipStream_t s) {
  const int nc = (int)g->circ.size();
  if (!bs_offsets) fail(QFLEX_E_INVALID, "NULL argument");
  if (g->max_pieces > dev::kMaxPiecesGrad)
    fail(QFLEX_E_UNSUPPORTED, "gradients support at most " +
                                  std::to_string(dev::kMaxPiecesGrad) + " gates per qubit");
  const int no = (int)g->circ[0].plan.open.size();
  const int64_t namp = int64_t(1) << no;
  const int64_t total_bs = bs_offsets[nc];
  const int64_t total_amp = total_bs * namp;
  // ---- host checks, slice selection and output-offset upload
  g->amps_dev.reserve(sizeof(double2) * std::max<int64_t>(total_amp, 1));
  double2* amps = static_cast<double2*>(g->amps_dev.p);
  const std::vector<std::vector<int64_t>> sel =
      prepare_call(g, bits, bs_offsets, fidelity, seed, slice_ids, slice_offsets, amps, s);
  // With one slice per circuit, the forward pass that keeps the intermediates for the reverse
  // sweep already yields the amplitudes (and, batch by batch, the linear-XEB cotangent), so no
  // separate amplitude pass runs.  Otherwise every slice's cotangent needs the full sum first.
  bool fused = true;
  for (int c = 0; c < nc; ++c)
    fused = fused && sel[c].size() == 1 && !g->circ[c].plan.result.qubit;
  qflex_stats fwd{};
  if (!fused) {
    contract(g, bits, bs_offsets, fidelity, seed, slice_ids, slice_offsets,
             reinterpret_cast<double*>(amps), QFLEX_OUT_DEVICE, s);
    fwd = g->last;
  }
  // ---- cotangent of the amplitudes, kept as dL/d(conj psi)
  g->gbar.reserve(sizeof(double2) * std::max<int64_t>(total_amp, 1));
  double2* gbar = static_cast<double2*>(g->gbar.p);
  g->xeb.reserve(sizeof(double) * std::max(nc, 1));
  double* xeb_sum = static_cast<double*>(g->xeb.p);
  std::vector<double> scale(nc, 0.0);
  if (cot) {
    // the caller's cotangent is dL/dRe + i dL/dIm = 2 dL/d(conj amp); keep dL/d(conj amp)
    if (total_amp > 0) {
      QHIPG(hipMemcpyAsync(gbar, cot, sizeof(double2) * total_amp,
                           cot_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
      dev::fill_zero(xeb_sum, nc, s);
      dev::xeb_cotangent(gbar, total_amp, 0.5, gbar, xeb_sum, s);
    }
  } else {
    for (int c = 0; c < nc; ++c) {
      const int64_t m = (bs_offsets[c + 1] - bs_offsets[c]) * namp;
      if (m) scale[c] = std::ldexp(1.0, g->circ[c].model.n) / (double)m;  // linear XEB 2^n/m
    }
  }
  // ---- FP64 cotangents of the qubit tensors and of the piece matrices
  g->tbar.reserve(sizeof(double2) * std::max<int64_t>(g->grid_elems, 1));
  g->pbar.reserve(sizeof(double2) * 4 * std::max<int64_t>(g->n_mats, 1));
  double2* tbar = static_cast<double2*>(g->tbar.p);
  double2* pbar = static_cast<double2*>(g->pbar.p);
  // slices (same rule as the forward call) and output-offset table layout
  std::vector<int64_t> offs_base(nc + 1, 0);
  for (int c = 0; c < nc; ++c)
    offs_base[c + 1] = offs_base[c] + (bs_offsets[c + 1] - bs_offsets[c]) * g->circ[c].model.n;
  const int64_t* offs_dev = static_cast<const int64_t*>(g->offs.p);
  size_t free_b = 0, total_b = 0;
  QHIPG(hipMemGetInfo(&free_b, &total_b));
  qflex_stats st = fwd;
  const int64_t tuned0 = g->n_tuned - fwd.n_tuned;
  // ---- per circuit: memory layout (checkpoints, one segment's values and cotangents, two
  // product scratches), bit-strings per batch and the split-K workspace of its products.
  // Everything is reserved before the first launch, so that the launches can be captured.
  std::vector<int64_t> batch(nc, 1), ws_elems(nc, 0);
  size_t arena_need = sizeof(float2), ws_need_all = 0;
  for (int c = 0; c < nc; ++c) {
    CircuitState& cs = g->circ[c];
    const Plan& P = cs.plan;
    const int64_t nbs = bs_offsets[c + 1] - bs_offsets[c];
    if (nbs == 0) continue;
    if (!cs.grad_layout_ready) {
      cs.grad_layout = make_grad_layout(P, namp);
      cs.grad_layout_ready = true;
    }
    const double per = 8.0 * (double)cs.grad_layout.elems;
    int64_t B = (int64_t)std::max(
        1.0, std::floor(std::min(0.5 * ((double)free_b + g->grad_arena.bytes),
                                 96.0 * (1ull << 30)) / per));
    B = std::min<int64_t>(std::min<int64_t>(B, nbs), 1024);
    batch[c] = B;
    arena_need = std::max(arena_need, sizeof(float2) * (size_t)(cs.grad_layout.elems * B));
    // split-K workspace for the products of this circuit (forward, Xbar and Ybar shapes) at
    // the batch sizes it runs (full batches and the last, partial one), for every kernel
    // variant that fits: the autotuner must time each one as it would run
    int64_t ws_need = 0;
    for (int64_t nbv : {B, nbs % B}) {
      if (nbv <= 0) continue;
      for (const Step& stp : P.steps) {
        const int64_t M = int64_t(1) << stp.mb, K = int64_t(1) << stp.kb,
                      N = int64_t(1) << stp.nb;
        const int64_t shapes[3][3] = {{M, N, K}, {M, K, N}, {K, N, M}};  // (rows, cols, depth)
        for (const auto& sh : shapes) {
          dev::Gemm q;
          q.M = sh[0];
          q.N = sh[1];
          q.K = sh[2];
          q.batch = (int)nbv;
          for (int v = 0; v < dev::kGemmVariants; ++v) {
            if (!dev::gemm_variant_fits(q, v)) continue;
            q.force_variant = v;
            ws_need = std::max(ws_need, dev::gemm_splitk_elems(q));
          }
        }
      }
    }
    ws_elems[c] = ws_need;
    ws_need_all = std::max(ws_need_all, sizeof(float2) * (size_t)ws_need);
  }
  g->grad_arena.reserve(arena_need);
  if (ws_need_all) g->splitk_ws.reserve(ws_need_all);
  // the host's copies of the piece cotangents and of the cross-entropy sums
  const size_t host_pbar = sizeof(double2) * 4 * std::max<int64_t>(g->n_mats, 1);
  g->grad_host.reserve(host_pbar + sizeof(double) * std::max(nc, 1));
  double2* hp = static_cast<double2*>(g->grad_host.p);
  double* hx = reinterpret_cast<double*>(static_cast<char*>(g->grad_host.p) + host_pbar);
  // ---- every launch of the call (captured once and replayed in graph mode)
  auto enqueue = [&] {
    if (fused) dev::fill_zero(reinterpret_cast<double*>(amps), 2 * total_amp, s);
    if (!cot) {
      dev::fill_zero(xeb_sum, nc, s);
      if (!fused)
        for (int c = 0; c < nc; ++c) {
          const int64_t m = (bs_offsets[c + 1] - bs_offsets[c]) * namp;
          if (m)
            dev::xeb_cotangent(amps + bs_offsets[c] * namp, m, scale[c],
                               gbar + bs_offsets[c] * namp, xeb_sum + c, s);
        }
    }
    dev::fill_zero(reinterpret_cast<double*>(tbar), 2 * g->grid_elems, s);
    dev::fill_zero(reinterpret_cast<double*>(pbar), 8 * g->n_mats, s);
    for (int c = 0; c < nc; ++c) {
      CircuitState& cs = g->circ[c];
      const Plan& P = cs.plan;
      const int64_t nbs = bs_offsets[c + 1] - bs_offsets[c];
      if (nbs == 0) continue;
      const std::vector<int64_t>& slices = sel[c];
      const GradLayout& GL = cs.grad_layout;
      const std::vector<int64_t>& voff = GL.voff;
      const std::vector<int64_t>& coff = GL.coff;
      const int64_t s1off = GL.s1off, s2off = GL.s2off;
      const int64_t B = batch[c];
      float2* ar = static_cast<float2*>(g->grad_arena.p);
      const int64_t ws_need = ws_elems[c];
      float2* splitk_ws = ws_need ? static_cast<float2*>(g->splitk_ws.p) : nullptr;
      // forward products whose intermediate x the MFMA rows kernel reads in its own storage order
      // (decided at grid build), kept to K >= 256 so that the backward X^T Zbar reads it the same
      // way on that kernel (its rows are then a multiple of 256)
      auto gathered = [&](size_t k) {
        return !cs.gather_x.empty() && cs.gather_x[k] && P.steps[k].kb >= 8;
      };
      // permutations routing each product cotangent back to its operand's storage order
      std::vector<dev::PermTile> rx(P.steps.size()), ry(P.steps.size());
      std::vector<PermDesc> dx(P.steps.size()), dy(P.steps.size());
      for (size_t k = 0; k < P.steps.size(); ++k) {
        const Step& stp = P.steps[k];
        dx[k] = make_perm_desc(cat(stp.mlab, stp.klab), stp.x_in);
        dy[k] = make_perm_desc(cat(stp.klab, stp.nlab), stp.y_in);
        if (!stp.x.qubit) rx[k] = dev::make_perm_tile(dx[k].nbits, dx[k].perm.data());
        if (!stp.y.qubit) ry[k] = dev::make_perm_tile(dy[k].nbits, dy[k].perm.data());
      }
      const float2* grid = g->grid + cs.grid_offset;
      double2* tgrid = tbar + cs.grid_offset;
      const int ncut = (int)P.cuts.size();
      for (int64_t b0 = 0; b0 < nbs; b0 += B) {
        const int nb = (int)std::min<int64_t>(B, nbs - b0);
        std::vector<int64_t> digit(ncut, 0);
        auto view = [&](const Operand& o) {
          GView v;
          if (o.qubit) {
            const QubitLayout& L = P.qubits[o.id];
            v.base = grid + cs.qubit_offset[o.id];
            for (auto& cshift : L.cut_shift) v.add += digit[cshift.first] << cshift.second;
            if (L.out_shift >= 0) v.off = offs_dev + offs_base[c] + (int64_t)o.id * nbs + b0;
          } else {
            v.base = ar + voff[o.id] * B;
            v.bs = P.nodes[o.id].elems();
          }
          return v;
        };
        auto nodev = [&](int id) {
          GView v;
          v.base = ar + voff[id] * B;
          v.bs = P.nodes[id].elems();
          return v;
        };
        auto route = [&](const Operand& o, const float2* src, const PermDesc& d,
                         const dev::PermTile& t) {
          if (o.qubit) {
            const QubitLayout& L = P.qubits[o.id];
            int64_t add = cs.qubit_offset[o.id];
            for (auto& cshift : L.cut_shift) add += digit[cshift.first] << cshift.second;
            const int64_t* off =
                L.out_shift >= 0 ? offs_dev + offs_base[c] + (int64_t)o.id * nbs + b0 : nullptr;
            std::vector<int8_t> p8(d.perm.begin(), d.perm.end());
            g->prof.begin("scatter_add_perm", 0,
                          24.0 * (double)(int64_t(1) << d.nbits) * nb, s);
            dev::scatter_add_perm(src, d.nbits, p8.data(), nb, tgrid, off, add, s);
            g->prof.end(s);
          } else {
            g->prof.begin("permute", 0, 16.0 * (double)(int64_t(1) << d.nbits) * nb, s);
            dev::permute(src, ar + coff[o.id] * B, nb, t, s);
            g->prof.end(s);
            ++st.n_permute;
          }
        };
        for (int64_t sid : slices) {
          int64_t rem = sid;
          for (int ct = ncut - 1; ct >= 0; --ct) {
            digit[ct] = rem & ((int64_t(1) << P.cut_bits[ct]) - 1);
            rem >>= P.cut_bits[ct];
          }
          // forward product of step k: its output (and a permuted copy of an operand) go to the
          // step's place in the layout, a checkpoint's own or the segment area's
          auto forward_step = [&](size_t k) {
            const Step& stp = P.steps[k];
            GView x = view(stp.x), y = view(stp.y);
            const bool gx = gathered(k);
            if (stp.scratch_x >= 0 && !gx) {
              float2* dst = ar + voff[stp.scratch_x] * B;
              g->prof.begin("permute", 0,
                            16.0 * (double)P.nodes[stp.scratch_x].elems() * nb, s);
              dev::permute(x.base, dst, nb, cs.px[k], s);
              g->prof.end(s);
              x = nodev(stp.scratch_x);
            }
            if (stp.scratch_y >= 0) {
              float2* dst = ar + voff[stp.scratch_y] * B;
              g->prof.begin("permute", 0,
                            16.0 * (double)P.nodes[stp.scratch_y].elems() * nb, s);
              dev::permute(y.base, dst, nb, cs.py[k], s);
              g->prof.end(s);
              y = nodev(stp.scratch_y);
            }
            dev::Gemm gm;
            gm.A = x.base;
            gm.a_off = x.off;
            gm.a_bs = x.bs;
            gm.a_add = x.add;
            gm.B = y.base;
            gm.b_off = y.off;
            gm.b_bs = y.bs;
            gm.b_add = y.add;
            gm.C = ar + voff[stp.out] * B;
            gm.c_bs = P.nodes[stp.out].elems();
            gm.M = int64_t(1) << stp.mb;
            gm.K = int64_t(1) << stp.kb;
            gm.N = int64_t(1) << stp.nb;
            gm.ta = stp.ta;
            gm.tb = stp.tb;
            gm.lda = stp.ta ? gm.M : gm.K;
            gm.ldb = stp.tb ? gm.K : gm.N;
            gm.ldc = gm.N;
            gm.batch = nb;
            gm.ws = splitk_ws;
            gm.ws_elems = ws_need;
            if (gx) {  // x in its own storage order, on the MFMA rows kernel
              gm.gather = true;
              gm.ga = cs.gx[k];
              gm.ta = 0;
              gm.lda = gm.K;
              gm.force_variant = 8;
            } else {
              gm.force_variant = cs.tuned_grad[3 * k + 0];
              if (gm.force_variant < 0 && g->autotune)
                gm.force_variant = cs.tuned_grad[3 * k + 0] = tune_gemm(g, s, gm);
            }
            g->prof.begin(dev::gemm_name(gm), stp.flops() * nb,
                          8.0 * nb * (double)(gm.M * gm.K + gm.K * gm.N + gm.M * gm.N), s);
            dev::gemm(gm, s);
            g->prof.end(s);
            st.flops += stp.flops() * nb;
            ++st.n_gemm;
          };
          // forward: the checkpoints and the last segment stay; the other segments' own
          // intermediates are overwritten by the next segment's
          for (size_t k = 0; k < P.steps.size(); ++k) forward_step(k);
          if (fused) {  // this batch's amplitudes (its only slice), then its XEB cotangent
            const Node& rn = P.nodes[P.result.id];
            double2* ab = amps + (bs_offsets[c] + b0) * namp;
            dev::accumulate(ar + voff[P.result.id] * B, nullptr, rn.elems(), 0, namp,
                            g->bidx + cs.bidx_offset, ab, namp, nb, s);
            if (!cot)
              dev::xeb_cotangent(ab, nb * namp, scale[c], gbar + (bs_offsets[c] + b0) * namp,
                                 xeb_sum + c, s);
          }
          // seed: cotangent of the result = conj(gbar) of this batch's amplitudes
          const double2* gb = gbar + (bs_offsets[c] + b0) * namp;
          if (P.result.qubit) {
            float2* tmp = ar + s1off * B;
            dev::seed_cotangent(gb, g->bidx + cs.bidx_offset, namp, namp, nb, tmp, s);
            const QubitLayout& L = P.qubits[P.result.id];
            PermDesc idp;
            idp.nbits = L.free_bits();
            idp.perm.resize(idp.nbits);
            std::iota(idp.perm.begin(), idp.perm.end(), 0);
            route(P.result, tmp, idp, dev::PermTile{});
            continue;
          }
          dev::seed_cotangent(gb, g->bidx + cs.bidx_offset, namp, namp, nb,
                              ar + coff[P.result.id] * B, s);
          // reverse sweep, segment by segment from the last: each one but the last is first
          // recomputed from the checkpoints and the qubit tensors
          for (size_t si = GL.segs.size(); si-- > 0;) {
            if (si + 1 < GL.segs.size())
              for (int k = GL.segs[si].first; k < GL.segs[si].second; ++k) forward_step(k);
            for (size_t kk = GL.segs[si].second; kk-- > (size_t)GL.segs[si].first;) {
              const Step& stp = P.steps[kk];
              const int64_t M = int64_t(1) << stp.mb, K = int64_t(1) << stp.kb,
                            N = int64_t(1) << stp.nb;
              const bool gx = gathered(kk);
              GView x = stp.scratch_x >= 0 && !gx ? nodev(stp.scratch_x) : view(stp.x);
              GView y = stp.scratch_y >= 0 ? nodev(stp.scratch_y) : view(stp.y);
              const float2* zbar = ar + coff[stp.out] * B;
              float2* xbar = ar + s1off * B;  // [M][K]
              float2* ybar = ar + s2off * B;  // [K][N]
              dev::Gemm g1;  // Xbar = Zbar Y'^T
              g1.A = zbar;
              g1.a_bs = M * N;
              g1.lda = N;
              g1.B = y.base;
              g1.b_off = y.off;
              g1.b_bs = y.bs;
              g1.b_add = y.add;
              g1.tb = stp.tb ? 0 : 1;
              g1.M = M;
              g1.N = K;
              g1.K = N;
              g1.ldb = g1.tb ? N : K;
              g1.C = xbar;
              g1.c_bs = M * K;
              g1.ldc = K;
              g1.batch = nb;
              g1.ws = splitk_ws;
              g1.ws_elems = ws_need;
              g1.force_variant = cs.tuned_grad[3 * kk + 1];
              if (g1.force_variant < 0 && g->autotune)
                g1.force_variant = cs.tuned_grad[3 * kk + 1] = tune_gemm(g, s, g1);
              // Xbar of an intermediate x goes straight to x's cotangent in x's storage order
              // when its product runs on an MFMA tile (the tile writes through the bit-deposit
              // maps of that order; x is consumed by this step only, so nothing else writes
              // there): no scratch copy, no routing pass
              const bool xbar_direct =
                  !stp.x.qubit && dev::gemm_scatter_variant(dev::gemm_variant(g1));
              if (xbar_direct) {
                g1.scatter = true;
                g1.ws = nullptr;
                g1.ws_elems = 0;
                g1.C = ar + coff[stp.x.id] * B;
                g1.c_bs = P.nodes[stp.x.id].elems();
                // output (m, k): bit i of k and of m go where dx[kk] puts product-order bits
                // i and kb + i of cat(mlab, klab)
                const PermDesc& d = dx[kk];
                std::vector<int> dest(d.nbits, -1);
                for (int j = 0; j < d.nbits; ++j) dest[d.perm[j]] = j;
                g1.om.nn = stp.kb;
                g1.om.nm = stp.mb;
                for (int i = 0; i < stp.kb; ++i) g1.om.npos[i] = (int8_t)dest[i];
                for (int i = 0; i < stp.mb; ++i) g1.om.mpos[i] = (int8_t)dest[stp.kb + i];
              }
              g->prof.begin(dev::gemm_name(g1), stp.flops() * nb,
                            8.0 * nb * (double)(g1.M * g1.K + g1.K * g1.N + g1.M * g1.N), s);
              dev::gemm(g1, s);
              g->prof.end(s);
              dev::Gemm g2;  // Ybar = X'^T Zbar
              g2.A = x.base;
              g2.a_off = x.off;
              g2.a_bs = x.bs;
              g2.a_add = x.add;
              g2.ta = stp.ta ? 0 : 1;
              g2.M = K;
              g2.N = N;
              g2.K = M;
              g2.lda = g2.ta ? K : M;
              g2.B = zbar;
              g2.b_bs = M * N;
              g2.ldb = N;
              g2.C = ybar;
              g2.c_bs = K * N;
              g2.ldc = N;
              g2.batch = nb;
              g2.ws = splitk_ws;
              g2.ws_elems = ws_need;
              if (gx) {  // X^T read through the forward product's gather descriptor
                g2.gather = true;
                g2.ga = cs.gx[kk];
                g2.ta = 1;
                g2.lda = g2.M;
                g2.force_variant = 8;
              } else {
                g2.force_variant = cs.tuned_grad[3 * kk + 2];
                if (g2.force_variant < 0 && g->autotune)
                  g2.force_variant = cs.tuned_grad[3 * kk + 2] = tune_gemm(g, s, g2);
              }
              g->prof.begin(dev::gemm_name(g2), stp.flops() * nb,
                            8.0 * nb * (double)(g2.M * g2.K + g2.K * g2.N + g2.M * g2.N), s);
              dev::gemm(g2, s);
              g->prof.end(s);
              st.flops += 2.0 * stp.flops() * nb;
              st.n_gemm += 2;
              if (!xbar_direct) route(stp.x, xbar, dx[kk], rx[kk]);
              route(stp.y, ybar, dy[kk], ry[kk]);
            }
          }
        }
      }
      // reverse the time collapse of this circuit's qubits
      g->prof.begin("grid_adjoint", 0, 0, s);
      dev::grid_adjoint(static_cast<const dev::GridQubit*>(g->gq.p) + cs.qdesc_base, cs.model.n,
                        cs.max_nlb, static_cast<const dev::GridPiece*>(g->gpieces.p),
                        static_cast<const double2*>(g->gmats.p),
                        static_cast<const int32_t*>(g->gpos.p), tbar, pbar, s);
      g->prof.end(s);
    }
    // the piece cotangents and the cross-entropy sums to the host
    QHIPG(hipMemcpyAsync(hp, pbar, sizeof(double2) * 4 * g->n_mats, hipMemcpyDeviceToHost, s));
    if (!cot) QHIPG(hipMemcpyAsync(hx, xeb_sum, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
  };  // enqueue
  // ---- graph mode: with one slice per circuit every launch depends only on the call's shape
  // (bit-strings per circuit, their batching, the slices, whether a cotangent is given) and on
  // buffer addresses; the bit-strings travel in g->offs and the cotangent in gbar, both written
  // before the launches.  The first call tunes (eagerly), the next captures, later ones replay.
  const bool tuning = g->autotune && !g->grad_tuned;
  if (g->graph_mode && fused && !tuning) {
    hipStream_t gs = s;
    if (!s) {  // the null stream cannot capture: the grid's own stream, ordered by events
      if (!g->graph_stream) {
        QHIPG(hipStreamCreateWithFlags(&g->graph_stream, hipStreamNonBlocking));
        QHIPG(hipEventCreateWithFlags(&g->graph_in, hipEventDisableTiming));
        QHIPG(hipEventCreateWithFlags(&g->graph_out, hipEventDisableTiming));
      }
      QHIPG(hipEventRecord(g->graph_in, s));
      QHIPG(hipStreamWaitEvent(g->graph_stream, g->graph_in, 0));
      gs = g->graph_stream;
    }
    std::string key;
    const void* keyed[] = {g->grad_arena.p, g->splitk_ws.p, amps, gbar, xeb_sum, tbar, pbar,
                           g->offs.p, g->grad_host.p, gs};
    for (const void* p : keyed) key += std::to_string(reinterpret_cast<uintptr_t>(p)) + ",";
    key += cot ? "c" : "x";
    for (int c = 0; c < nc; ++c)
      key += "|" + std::to_string(bs_offsets[c + 1] - bs_offsets[c]) + ":" +
             std::to_string(batch[c]) + ":" + std::to_string(sel[c].empty() ? -1 : sel[c][0]);
    if (g->grad_graph_exec && key == g->grad_graph_key) {
      QHIPG(hipGraphLaunch(g->grad_graph_exec, gs));
      st = g->grad_graph_stats;
    } else {
      if (g->grad_graph_exec) {
        QHIPG(hipGraphExecDestroy(g->grad_graph_exec));
        g->grad_graph_exec = nullptr;
        g->grad_graph_key.clear();
      }
      const bool prof_was_on = g->prof.on;
      g->prof.on = false;  // no event records inside a graph
      const hipStream_t s_call = s;
      s = gs;
      QHIPG(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipGraph_t gr = nullptr;
      try {
        enqueue();
      } catch (...) {
        (void)hipStreamEndCapture(s, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        s = s_call;
        g->prof.on = prof_was_on;
        throw;
      }
      const hipError_t e = hipStreamEndCapture(s, &gr);
      s = s_call;
      g->prof.on = prof_was_on;
      if (e != hipSuccess || !gr) {
        if (gr) (void)hipGraphDestroy(gr);
        fail(QFLEX_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      }
      hipGraphExec_t ex = nullptr;
      const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (ei != hipSuccess)
        fail(QFLEX_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
      g->grad_graph_exec = ex;
      g->grad_graph_key = key;
      g->grad_graph_stats = st;
      QHIPG(hipGraphLaunch(ex, gs));
    }
    if (gs != s) {
      QHIPG(hipEventRecord(g->graph_out, gs));
      QHIPG(hipStreamWaitEvent(s, g->graph_out, 0));
    }
  } else {
    enqueue();
    if (g->autotune) g->grad_tuned = true;
  }
  QHIPG(hipStreamSynchronize(s));
  // ---- host: piece cotangents -> gate entries -> angles (FP64)
  std::vector<cdouble> gg;      // gate-entry gradients, PyTorch convention
  std::vector<double> gpar;     // [gates][2]
  std::vector<double> lossv(nc, std::nan(""));
  for (int c = 0; c < nc; ++c) {
    const CircuitState& cs = g->circ[c];
    const Model& m = cs.model;
    std::vector<std::vector<cdouble>> gb(m.gates.size());
    for (size_t gi = 0; gi < m.gates.size(); ++gi) gb[gi].assign(m.gates[gi].q1 < 0 ? 4 : 16, 0.0);
    for (int q = 0; q < m.n; ++q)
      for (const Piece& pc : m.timeline[q]) {
        const int mi = cs.mat_base + pc.mat;
        auto P = [&](int k, int e) { return cdouble(hp[4 * (mi + k) + e].x, hp[4 * (mi + k) + e].y); };
        const Gate& G = m.gates[pc.gate];
        if (G.q1 < 0) {
          for (int e = 0; e < 4; ++e) gb[pc.gate][e] += P(0, e);
        } else if (pc.hi_side) {
          const int rank = 1 << pc.kbits;
          for (int k = 0; k < rank; ++k) {
            const int i = rank == 2 ? k : k >> 1, j = rank == 2 ? k : k & 1;
            for (int a = 0; a < 2; ++a)
              for (int b = 0; b < 2; ++b) gb[pc.gate][(2 * i + a) * 4 + 2 * j + b] += P(k, 2 * a + b);
          }
        }
      }
    for (size_t gi = 0; gi < m.gates.size(); ++gi) {
      const Gate& G = m.gates[gi];
      std::vector<cdouble> d = gb[gi];
      if (G.q1 >= 0 && G.q0 > G.q1) {  // back from the |lo hi> basis to the gate's own order
        static const int sw[4] = {0, 2, 1, 3};
        for (int r = 0; r < 4; ++r)
          for (int t = 0; t < 4; ++t) d[r * 4 + t] = gb[gi][sw[r] * 4 + sw[t]];
      }
      double dth = 0, dph = 0;
      if (G.kind == QFLEX_G_FSIM) {
        const double cth = std::cos(G.theta), sth = std::sin(G.theta);
        const cdouble I(0, 1);
        // dG/dtheta and dG/dphi of fSim, entries (1,1),(1,2),(2,1),(2,2),(3,3)
        const cdouble dt5 = -sth, dt6 = -I * cth, dt9 = -I * cth, dt10 = -sth;
        const cdouble dp15 = -I * std::exp(-I * G.phi);
        dth = 2.0 * std::real(d[5] * dt5 + d[6] * dt6 + d[9] * dt9 + d[10] * dt10);
        dph = 2.0 * std::real(d[15] * dp15);
      }
      gpar.push_back(dth);
      gpar.push_back(dph);
      for (const cdouble& z : d) gg.push_back(2.0 * std::conj(z));  // dL/dRe + i dL/dIm
    }
    if (!cot && bs_offsets[c + 1] > bs_offsets[c]) lossv[c] = scale[c] * hx[c] - 1.0;
  }
  const hipMemcpyKind kind = out_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
  if (grad_gates && !gg.empty())
    QHIPG(hipMemcpyAsync(grad_gates, gg.data(), sizeof(cdouble) * gg.size(), kind, s));
  if (grad_params && !gpar.empty())
    QHIPG(hipMemcpyAsync(grad_params, gpar.data(), sizeof(double) * gpar.size(), kind, s));
  if (loss) QHIPG(hipMemcpyAsync(loss, lossv.data(), sizeof(double) * nc, kind, s));
  if (amps_out && total_amp > 0)
    QHIPG(hipMemcpyAsync(amps_out, amps, sizeof(double2) * total_amp,
                         out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  QHIPG(hipStreamSynchronize(s));
  if (g->prof.on) g->prof.resolve();
  st.n_tuned = g->n_tuned - tuned0;
  g->last = st;
}

}  // namespace qflex
