// C entry points: argument checks, status codes, thread-local error messages.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/qflex_kernels.h"
#include "api_internal.h"
#include "fused_plan.h"
#include "grid.h"

namespace {

thread_local std::string g_last_error;

qflex_status set_error(qflex_status s, const std::string& m) {
  g_last_error = m;
  return s;
}

template <class F>
qflex_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return QFLEX_OK;
  } catch (const qflex::Error& e) {
    return set_error(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return set_error(QFLEX_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(QFLEX_E_DEVICE, e.what());
  }
}

void release(qflex_grid* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  if (g->grid) (void)hipFree(g->grid);
  if (g->bidx) (void)hipFree(g->bidx);
  if (g->grid_split) (void)hipFree(g->grid_split);
  if (g->amax) (void)hipFree(g->amax);
  if (g->node_amax) (void)hipFree(g->node_amax);
  if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
  if (g->grad_graph_exec) (void)hipGraphExecDestroy(g->grad_graph_exec);
  if (g->graph_in) (void)hipEventDestroy(g->graph_in);
  for (hipEvent_t e : g->tune_ev)
    if (e) (void)hipEventDestroy(e);
  if (g->graph_out) (void)hipEventDestroy(g->graph_out);
  if (g->graph_stream) (void)hipStreamDestroy(g->graph_stream);
  g->split_scratch.release();
  g->split_cache.release();
  for (qflex::DevBuf* b : {&g->gq, &g->gpieces, &g->gmats, &g->gpos, &g->grad_arena, &g->tbar,
                           &g->pbar, &g->gbar, &g->amps_dev, &g->xeb, &g->splitk_ws,
                           &g->fs_buf})
    b->release();
  g->arena.release();
  g->amps64.release();
  g->offs.release();
  g->offs_host.release();
  g->grad_host.release();
  g->fused_prog.release();
  if (g->offs_done) (void)hipEventDestroy(g->offs_done);
  for (int k = 0; k < 2; ++k) {
    if (g->offs_pinned_done[k]) {
      (void)hipEventSynchronize(g->offs_pinned_done[k]);
      (void)hipEventDestroy(g->offs_pinned_done[k]);
    }
    g->offs_pinned[k].release();
  }
  g->prof.release();
  delete g;
}

void check_options(const qflex_options& o) {
  if (o.precision != QFLEX_PREC_C64 && o.precision != QFLEX_PREC_SPLIT_BF16 &&
      o.precision != QFLEX_PREC_SPLIT_FP16)
    qflex::fail(QFLEX_E_INVALID, "unknown precision");
  if (o.plan_kind < QFLEX_PLAN_AUTO || o.plan_kind > QFLEX_PLAN_CUT_SWEEP)
    qflex::fail(QFLEX_E_INVALID, "unknown plan_kind");
  if (o.bitstring_batch < 0) qflex::fail(QFLEX_E_INVALID, "bitstring_batch < 0");
  if (o.slice_mode != QFLEX_SLICES_RANDOM && o.slice_mode != QFLEX_SLICES_BLOCK)
    qflex::fail(QFLEX_E_INVALID, "unknown slice_mode");
  if (o.graph != 0 && o.graph != 1) qflex::fail(QFLEX_E_INVALID, "graph must be 0 or 1");
  if (o.autotune != 0 && o.autotune != 1) qflex::fail(QFLEX_E_INVALID, "autotune must be 0 or 1");
  if (o.fused < -1 || o.fused > 1) qflex::fail(QFLEX_E_INVALID, "fused must be -1, 0 or 1");
  if (o.fused == 1 && o.precision != QFLEX_PREC_C64)
    qflex::fail(QFLEX_E_INVALID, "the fused contraction runs in complex64 only");
}

}  // namespace

namespace qflex {

qflex_status run_guarded(const std::function<void()>& f) { return guarded(f); }

// Every check of the split product's arguments except the workspace's.
void gemm_split_c64_check(const void* A, const void* B, const void* C, int64_t M, int64_t N,
                          int64_t K, int32_t ta, int32_t tb, int64_t batch, int32_t precision) {
  if (!A || !B || !C) fail(QFLEX_E_INVALID, "NULL argument");
  if (precision != QFLEX_PREC_SPLIT_BF16 && precision != QFLEX_PREC_SPLIT_FP16)
    fail(QFLEX_E_INVALID, "precision must be QFLEX_PREC_SPLIT_BF16 or QFLEX_PREC_SPLIT_FP16");
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15)
    fail(QFLEX_E_INVALID, "A and B must be 16-byte aligned");
  const int mb = log2_exact(M), nb = log2_exact(N), kb = log2_exact(K);
  if (mb < 0 || nb < 0 || kb < 0) fail(QFLEX_E_INVALID, "M, N, K must be powers of two");
  if (!dev::gemm_split_ok(M, N, K) || mb + kb > 40 || nb + kb > 40)
    fail(QFLEX_E_INVALID, "shape too small or too large for the split product");
  if (batch < 1 || batch > 65535) fail(QFLEX_E_INVALID, "batch must be in [1, 65535]");
  if ((ta != 0 && ta != 1) || (tb != 0 && tb != 1)) fail(QFLEX_E_INVALID, "ta/tb must be 0 or 1");
}

// The split product on a workspace of the caller's (checked, then enqueued on st).
void gemm_split_c64_run(const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K,
                        int32_t ta, int32_t tb, int64_t batch, int32_t precision, int32_t tile,
                        void* workspace, int64_t workspace_bytes, hipStream_t st) {
  gemm_split_c64_check(A, B, C, M, N, K, ta, tb, batch, precision);
  if (tile != -1) {
    dev::GemmSplit shape;
    shape.M = M;
    shape.N = N;
    shape.K = K;
    if (tile < 0 || tile >= dev::kSplitTiles || !dev::gemm_split_tile_fits(shape, tile))
      fail(QFLEX_E_INVALID, "tile out of range or not fitting M, N");
  }
  if (!workspace) fail(QFLEX_E_INVALID, "NULL argument");
  if (workspace_bytes < qflex_gemm_split_workspace(M, N, K, batch))
    fail(QFLEX_E_INVALID, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) & 15)
    fail(QFLEX_E_INVALID, "workspace must be 16-byte aligned");
  const int mb = log2_exact(M), nb = log2_exact(N), kb = log2_exact(K);
  // bit permutation transposing [R][C] (rb, cb bits) into [C][R]
  auto transpose = [](int rb, int cb) {
    std::vector<int> p(rb + cb);
    for (int j = 0; j < rb + cb; ++j) p[j] = j < rb ? cb + j : j - rb;
    return p;
  };
  std::vector<int> pa(mb + kb), pbv(nb + kb);
  for (int j = 0; j < mb + kb; ++j) pa[j] = j;
  for (int j = 0; j < nb + kb; ++j) pbv[j] = j;
  if (ta) pa = transpose(kb, mb);   // stored [K][M] -> [M][K]
  if (!tb) pbv = transpose(kb, nb); // stored [K][N] -> [N][K]
  auto* slots = static_cast<uint64_t*>(workspace);
  auto* sa = reinterpret_cast<uint16_t*>(static_cast<char*>(workspace) + kSplitSlotBytes);
  auto* sb = sa + dev::kSplitValues * batch * M * K;
  const bool f16 = precision == QFLEX_PREC_SPLIT_FP16;
  if (f16) {  // the workspace holds anything: clear the slots (a fill kernel), then tag 1
    dev::fill_zero(reinterpret_cast<double*>(slots), 2, st);
    dev::absmax(static_cast<const float2*>(A), batch * M * K, slots, 1, st);
    dev::absmax(static_cast<const float2*>(B), batch * N * K, slots + 1, 1, st);
  }
  // A stored [M][K] is read by the product itself (identity gather), else permuted and split
  if (ta)
    dev::split_permute(static_cast<const float2*>(A), sa, batch,
                       dev::make_perm_tile(mb + kb, pa.data()), kb, f16 ? slots : nullptr, st);
  dev::split_permute(static_cast<const float2*>(B), sb, batch,
                     dev::make_perm_tile(nb + kb, pbv.data()), kb, f16 ? slots + 1 : nullptr, st);
  dev::GemmSplit g;
  if (f16) g.a_amax = slots, g.b_amax = slots + 1;
  if (!ta) {
    g.Ac = static_cast<const float2*>(A);
    g.ga.nm = mb;
    g.ga.nk = kb - 2;
    for (int i = 0; i < mb; ++i) g.ga.mpos[i] = (int8_t)(kb + i);
    for (int j = 0; j < kb - 2; ++j) g.ga.kpos[j] = (int8_t)(2 + j);
  }
  g.A = sa;
  g.B = sb;
  g.C = static_cast<float2*>(C);
  g.M = M;
  g.N = N;
  g.K = K;
  g.a_bs = M * K;
  g.b_bs = N * K;
  g.c_bs = M * N;
  g.batch = (int)batch;
  g.tile = tile;
  dev::gemm_split(g, st);
}

}  // namespace qflex

extern "C" {

qflex_status qflex_build_grid(const qflex_circuit* circuits, int32_t n_circuits,
                              const qflex_options* opt, void* stream, qflex_grid** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!circuits || !opt || !out) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (n_circuits < 1) qflex::fail(QFLEX_E_INVALID, "n_circuits must be >= 1");
    check_options(*opt);
    auto* g = new qflex_grid();
    try {
      g->precision = opt->precision;
      g->bitstring_batch = opt->bitstring_batch;
      g->slice_mode = opt->slice_mode;
      g->graph_mode = opt->graph != 0;
      g->autotune = opt->autotune != 0;
      g->fused_opt = opt->fused;
      for (int c = 0; c < n_circuits; ++c) {
        qflex::CircuitState cs;
        cs.model = qflex::build_model(circuits[c]);
        cs.plan = qflex::make_plan(cs.model, *opt);
        g->circ.push_back(std::move(cs));
      }
      int dev = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e != hipSuccess) qflex::fail(QFLEX_E_DEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
      g->device = dev;
      g->device_sig = qflex::device_signature(dev);
      qflex::build_grid_device(g, static_cast<hipStream_t>(stream));
    } catch (...) {
      release(g);
      throw;
    }
    *out = g;
  });
}

qflex_status qflex_update_gates(qflex_grid* g, int32_t circuit, const qflex_circuit* updated,
                                void* stream) {
  return guarded([&] {
    if (!g || !updated) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    qflex::update_gates(g, circuit, *updated, static_cast<hipStream_t>(stream));
  });
}

qflex_status qflex_num_slices(const qflex_grid* g, int32_t circuit, int64_t* total) {
  return guarded([&] {
    if (!g || !total) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (circuit < 0 || circuit >= (int)g->circ.size()) qflex::fail(QFLEX_E_INVALID, "bad circuit");
    *total = g->circ[circuit].plan.num_slices();
  });
}

qflex_status qflex_plan_cuts(const qflex_grid* g, int32_t circuit, int32_t* pairs,
                             int32_t max_cuts, int32_t* n_cuts) {
  return guarded([&] {
    if (!g || !n_cuts || (max_cuts > 0 && !pairs)) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (circuit < 0 || circuit >= (int)g->circ.size()) qflex::fail(QFLEX_E_INVALID, "bad circuit");
    const auto& cs = g->circ[circuit];
    *n_cuts = (int32_t)cs.plan.cuts.size();
    for (int i = 0; i < (int)cs.plan.cuts.size() && i < max_cuts; ++i) {
      pairs[2 * i] = cs.model.links[cs.plan.cuts[i]].lo;
      pairs[2 * i + 1] = cs.model.links[cs.plan.cuts[i]].hi;
    }
  });
}

qflex_status qflex_plan_describe(const qflex_circuit* circuit, const qflex_options* opt,
                                 char* buf, int64_t len, int64_t* needed) {
  return guarded([&] {
    if (!circuit || !opt) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    check_options(*opt);
    qflex::Model m = qflex::build_model(*circuit);
    qflex::Plan p = qflex::make_plan(m, *opt);
    std::string s = p.describe(m);
    // whether the plan fits the fused small-plan kernel (complex64 grids use it unless the
    // fused option is -1)
    s.insert(s.size() - 1, ",\"fused\":" + qflex::describe_fused(p, m));
    if (needed) *needed = (int64_t)s.size() + 1;
    if (buf && len > 0) {
      const size_t n = std::min<size_t>(s.size(), (size_t)len - 1);
      std::memcpy(buf, s.data(), n);
      buf[n] = '\0';
    }
  });
}

qflex_status qflex_contract_amplitudes(qflex_grid* g, const uint8_t* bits,
                                       const int64_t* bs_offsets, double fidelity,
                                       uint64_t slice_seed, const int64_t* slice_ids,
                                       const int64_t* slice_offsets, double* amps,
                                       int32_t amps_on_device, void* stream) {
  return guarded([&] {
    if (!g) qflex::fail(QFLEX_E_INVALID, "NULL grid");
    qflex::contract(g, bits, bs_offsets, fidelity, slice_seed, slice_ids, slice_offsets, amps,
                    amps_on_device, static_cast<hipStream_t>(stream));
  });
}

qflex_status qflex_contract_grad(qflex_grid* g, const uint8_t* bits, const int64_t* bs_offsets,
                                 double fidelity, uint64_t slice_seed, const int64_t* slice_ids,
                                 const int64_t* slice_offsets, const double* cotangent,
                                 int32_t cotangent_on_device, double* amps, double* grad_gates,
                                 double* grad_params, double* loss, int32_t out_on_device,
                                 void* stream) {
  return guarded([&] {
    if (!g) qflex::fail(QFLEX_E_INVALID, "NULL grid");
    qflex::contract_grad(g, bits, bs_offsets, fidelity, slice_seed, slice_ids, slice_offsets,
                         cotangent, cotangent_on_device, amps, grad_gates, grad_params, loss,
                         out_on_device != 0, static_cast<hipStream_t>(stream));
  });
}

qflex_status qflex_last_stats(const qflex_grid* g, qflex_stats* out) {
  return guarded([&] {
    if (!g || !out) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    *out = g->last;
  });
}

qflex_status qflex_set_profiling(qflex_grid* g, int32_t enable) {
  return guarded([&] {
    if (!g) qflex::fail(QFLEX_E_INVALID, "NULL grid");
    g->prof.on = enable != 0;
    g->prof.sums.clear();
  });
}

qflex_status qflex_profile_read(const qflex_grid* g, qflex_kernel_stat* out, int32_t max,
                                int32_t* n) {
  return guarded([&] {
    if (!g || !n || (max > 0 && !out)) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    *n = (int32_t)g->prof.sums.size();
    int i = 0;
    for (const auto& kv : g->prof.sums) {
      if (i >= max) break;
      qflex_kernel_stat& k = out[i++];
      std::memset(&k, 0, sizeof(k));
      std::strncpy(k.name, kv.first.c_str(), sizeof(k.name) - 1);
      k.launches = kv.second.launches;
      k.ms = kv.second.ms;
      k.flops = kv.second.flops;
      k.bytes = kv.second.bytes;
    }
  });
}

void qflex_grid_free(qflex_grid* g) { release(g); }

qflex_status qflex_permute_c64(const void* in, void* out, int32_t nbits, const int32_t* perm,
                               int64_t batch, void* stream) {
  return guarded([&] {
    if (!in || !out || !perm) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (nbits < 1 || nbits > 40) qflex::fail(QFLEX_E_INVALID, "nbits must be in [1, 40]");
    if (batch < 1 || batch > 65535) qflex::fail(QFLEX_E_INVALID, "batch must be in [1, 65535]");
    std::vector<int> p(perm, perm + nbits), seen(nbits, 0);
    for (int v : p) {
      if (v < 0 || v >= nbits || seen[v]) qflex::fail(QFLEX_E_INVALID, "perm is not a permutation");
      seen[v] = 1;
    }
    const auto t = qflex::dev::make_perm_tile(nbits, p.data());
    qflex::dev::permute(static_cast<const float2*>(in), static_cast<float2*>(out), batch, t,
                        static_cast<hipStream_t>(stream));
  });
}

static qflex::dev::Gemm dense_gemm(int64_t M, int64_t N, int64_t K, int32_t ta, int32_t tb,
                                   int64_t batch) {
  qflex::dev::Gemm g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.ta = ta;
  g.tb = tb;
  g.lda = ta ? M : K;
  g.ldb = tb ? K : N;
  g.ldc = N;
  g.a_bs = M * K;
  g.b_bs = K * N;
  g.c_bs = M * N;
  g.batch = (int)batch;
  return g;
}

int64_t qflex_gemm_c64_workspace(int64_t M, int64_t N, int64_t K, int64_t batch) {
  if (M < 1 || N < 1 || K < 1 || batch < 1 || batch > 65535) return 0;
  return (int64_t)sizeof(float) * 2 * qflex::dev::gemm_splitk_elems(dense_gemm(M, N, K, 0, 0, batch));
}

qflex_status qflex_gemm_c64(const void* A, const void* B, void* C, int64_t M, int64_t N,
                            int64_t K, int32_t ta, int32_t tb, int64_t batch, void* workspace,
                            int64_t workspace_bytes, void* stream) {
  return guarded([&] {
    if (!A || !B || !C) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (workspace_bytes < 0) qflex::fail(QFLEX_E_INVALID, "negative workspace size");
    if (M < 1 || N < 1 || K < 1) qflex::fail(QFLEX_E_INVALID, "M, N, K must be >= 1");
    if (batch < 1 || batch > 65535) qflex::fail(QFLEX_E_INVALID, "batch must be in [1, 65535]");
    if ((ta != 0 && ta != 1) || (tb != 0 && tb != 1)) qflex::fail(QFLEX_E_INVALID, "ta/tb must be 0 or 1");
    qflex::dev::Gemm g = dense_gemm(M, N, K, ta, tb, batch);
    g.A = static_cast<const float2*>(A);
    g.B = static_cast<const float2*>(B);
    g.C = static_cast<float2*>(C);
    if (workspace) {
      g.ws = static_cast<float2*>(workspace);
      g.ws_elems = workspace_bytes / (int64_t)sizeof(float2);
    }
    if (qflex::dev::gemm_variant(g) > 0 &&
        ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15))
      qflex::fail(QFLEX_E_INVALID, "A and B must be 16-byte aligned");
    qflex::dev::gemm(g, static_cast<hipStream_t>(stream));
  });
}

int64_t qflex_gemm_split_workspace(int64_t M, int64_t N, int64_t K, int64_t batch) {
  if (M < 1 || N < 1 || K < 1 || batch < 1) return 0;
  return qflex::kSplitSlotBytes +
         (int64_t)sizeof(uint16_t) * qflex::dev::kSplitValues * batch * (M * K + N * K);
}


qflex_status qflex_gemm_split_c64(const void* A, const void* B, void* C, int64_t M, int64_t N,
                                  int64_t K, int32_t ta, int32_t tb, int64_t batch,
                                  int32_t precision, void* workspace, int64_t workspace_bytes,
                                  void* stream) {
  return guarded([&] {
    qflex::gemm_split_c64_run(A, B, C, M, N, K, ta, tb, batch, precision, -1, workspace,
                              workspace_bytes, static_cast<hipStream_t>(stream));
  });
}

qflex_status qflex_gemm_split_c64_tile(const void* A, const void* B, void* C, int64_t M,
                                       int64_t N, int64_t K, int32_t ta, int32_t tb,
                                       int64_t batch, int32_t precision, int32_t tile,
                                       void* workspace, int64_t workspace_bytes, void* stream) {
  return guarded([&] {
    qflex::gemm_split_c64_run(A, B, C, M, N, K, ta, tb, batch, precision, tile, workspace,
                              workspace_bytes, static_cast<hipStream_t>(stream));
  });
}

int32_t qflex_gemm_variant(int64_t M, int64_t N, int64_t K) {
  qflex::dev::Gemm g;
  g.M = M;
  g.N = N;
  g.K = K;
  return qflex::dev::gemm_variant(g);
}

qflex_status qflex_select_slices(int64_t total, double fidelity, uint64_t seed, int32_t mode,
                                 int64_t* ids, int64_t max_ids, int64_t* n) {
  return guarded([&] {
    if (!n || (max_ids > 0 && !ids)) qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (total < 1 || total > (int64_t(1) << 32)) qflex::fail(QFLEX_E_INVALID, "total out of range");
    const auto v = qflex::select_slices(total, fidelity, seed, mode);
    *n = (int64_t)v.size();
    for (int64_t i = 0; i < (int64_t)v.size() && i < max_ids; ++i) ids[i] = v[i];
  });
}

qflex_status qflex_frugal_sample(const double* amps, int64_t n_batch, int64_t batch_len,
                                 const int32_t* order, const double* u, int32_t n_c,
                                 int32_t n_qubits, double m, int32_t* accepted, double* partial,
                                 double* tail, void* stream) {
  return guarded([&] {
    if (!tail || (n_batch > 0 && (!amps || !accepted || !partial || (n_c > 0 && (!order || !u)))))
      qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (n_batch < 0 || batch_len < 1 || n_c < 0)
      qflex::fail(QFLEX_E_INVALID, "need n_batch >= 0, batch_len >= 1, n_c >= 0");
    if (n_qubits < 1 || n_qubits > 1000) qflex::fail(QFLEX_E_INVALID, "n_qubits out of range");
    if (!(m > 0.0) || !std::isfinite(m)) qflex::fail(QFLEX_E_INVALID, "M must be finite and > 0");
    qflex::dev::frugal_sample(reinterpret_cast<const double2*>(amps), n_batch, batch_len, order,
                              u, n_c, n_qubits, m, accepted, partial, tail,
                              static_cast<hipStream_t>(stream));
  });
}

qflex_status qflex_fidelity_samples(qflex_grid* g, const uint8_t* closed_bits, int64_t n_batch,
                                    const double* coins, double fidelity,
                                    const uint8_t* uniform_bits, const int32_t* order,
                                    const double* u, int32_t n_c, double m, uint8_t* samples,
                                    int8_t* status, void* stream) {
  return guarded([&] {
    if (!g) qflex::fail(QFLEX_E_INVALID, "NULL grid");
    if (g->circ.size() != 1) qflex::fail(QFLEX_E_INVALID, "the grid must hold one circuit");
    if (n_batch < 0 || n_c < 0) qflex::fail(QFLEX_E_INVALID, "need n_batch >= 0 and n_c >= 0");
    if (n_batch > 0 && (!closed_bits || !coins || !uniform_bits || !samples || !status ||
                        (n_c > 0 && (!order || !u))))
      qflex::fail(QFLEX_E_INVALID, "NULL argument");
    if (!(fidelity >= 0.0 && fidelity <= 1.0))
      qflex::fail(QFLEX_E_INVALID, "fidelity must be in [0, 1]");
    if (!(m > 0.0) || !std::isfinite(m)) qflex::fail(QFLEX_E_INVALID, "M must be finite and > 0");
    const qflex::CircuitState& cs = g->circ[0];
    const int n = cs.model.n;
    const std::vector<int>& open = cs.plan.open;
    const int no = (int)open.size();
    const int64_t blen = int64_t(1) << no;
    // the batches that get an exact sample, and their rows of every input
    std::vector<int64_t> exact;
    for (int64_t b = 0; b < n_batch; ++b)
      if (coins[b] < fidelity) exact.push_back(b);
    const int64_t ne = (int64_t)exact.size();
    std::vector<uint8_t> eb((size_t)(ne * n));
    std::vector<int32_t> eo((size_t)(ne * n_c));
    std::vector<double> eu((size_t)(ne * n_c));
    for (int64_t i = 0; i < ne; ++i) {
      const int64_t b = exact[i];
      std::memcpy(&eb[i * n], closed_bits + b * n, (size_t)n);
      for (int j = 0; j < n_c; ++j) {
        const int32_t v = order[b * n_c + j];
        if (v < 0 || v >= blen)
          qflex::fail(QFLEX_E_INVALID, "order holds a value outside [0, 2^n_open)");
        eo[i * n_c + j] = v;
        eu[i * n_c + j] = u[b * n_c + j];
      }
    }
    // open qubits' bits of the exact batches do not matter: the contraction leaves them open
    for (int64_t i = 0; i < ne; ++i)
      for (int q : open) eb[i * n + q] = 0;
    std::vector<int32_t> acc((size_t)ne);
    if (ne > 0) {
      const hipStream_t st = static_cast<hipStream_t>(stream);
      auto up = [](int64_t bytes) { return (bytes + 255) & ~int64_t(255); };
      const int64_t b_amps = up(16 * ne * blen), b_ord = up(4 * ne * std::max(n_c, 1)),
                    b_u = up(8 * ne * std::max(n_c, 1)), b_acc = up(4 * ne), b_part = up(8 * ne);
      g->fs_buf.reserve((size_t)(b_amps + b_ord + b_u + b_acc + b_part + 256));
      char* base = static_cast<char*>(g->fs_buf.p);
      double* amps = reinterpret_cast<double*>(base);
      int32_t* d_ord = reinterpret_cast<int32_t*>(base + b_amps);
      double* d_u = reinterpret_cast<double*>(base + b_amps + b_ord);
      int32_t* d_acc = reinterpret_cast<int32_t*>(base + b_amps + b_ord + b_u);
      double* d_part = reinterpret_cast<double*>(base + b_amps + b_ord + b_u + b_acc);
      double* d_tail = reinterpret_cast<double*>(base + b_amps + b_ord + b_u + b_acc + b_part);
      const int64_t offs[2] = {0, ne};
      qflex::contract(g, eb.data(), offs, 1.0, 0, nullptr, nullptr, amps, QFLEX_OUT_DEVICE, st);
      auto check = [](hipError_t e, const char* what) {
        if (e != hipSuccess)
          qflex::fail(QFLEX_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
      };
      if (n_c > 0) {
        check(hipMemcpyAsync(d_ord, eo.data(), 4 * ne * n_c, hipMemcpyHostToDevice, st), "upload");
        check(hipMemcpyAsync(d_u, eu.data(), 8 * ne * n_c, hipMemcpyHostToDevice, st), "upload");
      }
      qflex::dev::frugal_sample(reinterpret_cast<const double2*>(amps), ne, blen, d_ord, d_u, n_c,
                                n, m, d_acc, d_part, d_tail, st);
      check(hipMemcpyAsync(acc.data(), d_acc, 4 * ne, hipMemcpyDeviceToHost, st), "download");
      check(hipStreamSynchronize(st), "stream");
    }
    // compose: uniform samples by default; an exact batch writes its accepted open value into
    // the open qubits (the first open qubit most significant)
    std::memcpy(samples, uniform_bits, (size_t)(n_batch * n));
    std::memset(status, 0, (size_t)n_batch);
    for (int64_t i = 0; i < ne; ++i) {
      const int64_t b = exact[i];
      if (acc[i] < 0) {
        status[b] = -1;
        continue;
      }
      std::memcpy(samples + b * n, closed_bits + b * n, (size_t)n);
      for (int t = 0; t < no; ++t) samples[b * n + open[t]] = (uint8_t)((acc[i] >> (no - 1 - t)) & 1);
      status[b] = 1;
    }
  });
}

const char* qflex_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
