// Executor: builds the device grid and runs a plan over bit-strings and slices.
//
// Loop nest (paper, SI A): for each batch of bit-strings, for each selected slice in
// ascending id order, re-run only the steps whose result depends on a cut whose value changed
// since the previous slice; every other intermediate is reused from device memory.  The last
// step's result is added into an FP64 amplitude accumulator after every slice.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <set>

#include "fused_plan.h"
#include "grid.h"

namespace qflex {

#define QHIP(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      fail(e_ == hipErrorOutOfMemory ? QFLEX_E_NOMEM : QFLEX_E_DEVICE,                      \
           std::string(#expr) + ": " + hipGetErrorString(e_));                              \
  } while (0)

void DevBuf::reserve(size_t n) {
  if (n <= bytes) return;
  if (p) {
    QHIP(hipDeviceSynchronize());
    QHIP(hipFree(p));
    p = nullptr;
    bytes = 0;
  }
  QHIP(hipMalloc(&p, n));
  bytes = n;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void HostPinned::reserve(size_t n) {
  if (n <= bytes) return;
  if (p) QHIP(hipHostFree(p));
  p = nullptr;
  bytes = 0;
  QHIP(hipHostMalloc(&p, n, hipHostMallocDefault));
  bytes = n;
}

void HostPinned::release() {
  if (p) (void)hipHostFree(p);
  p = nullptr;
  bytes = 0;
}

// ------------------------------------------------------------------------------ profiler
hipEvent_t Profiler::take() {
  if (used == pool.size()) {
    hipEvent_t e;
    QHIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  return pool[used++];
}

void Profiler::begin(const char* name, double flops, double bytes, hipStream_t s) {
  if (!on) return;
  Rec r{name, take(), take(), flops, bytes};
  QHIP(hipEventRecord(r.a, s));
  pending.push_back(r);
}

void Profiler::end(hipStream_t s) {
  if (!on) return;
  QHIP(hipEventRecord(pending.back().b, s));
}

void Profiler::resolve() {
  for (const Rec& r : pending) {
    float ms = 0;
    QHIP(hipEventElapsedTime(&ms, r.a, r.b));
    Sum& x = sums[r.name];
    x.launches += 1;
    x.ms += ms;
    x.flops += r.flops;
    x.bytes += r.bytes;
  }
  pending.clear();
  used = 0;
}

void Profiler::release() {
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
  pending.clear();
  used = 0;
}

// ------------------------------------------------------------------------------ grid build
void prepare_split(qflex_grid* g, hipStream_t s);
void split_qubits(qflex_grid* g, int c, hipStream_t s);
void prepare_fused(qflex_grid* g, hipStream_t s);

// A complex64 tall-skinny product whose intermediate x would be permuted first: the MFMA rows
// kernel reads x in its own storage order instead, when x's 2 lowest storage labels are
// contracted ones and x already stores the contracted labels in the product's order (so y and
// the output keep their layouts).  Such products (N <= 16) never run as split products.
static void c64_gather(const Step& st, dev::SplitGather& ga, char& use) {
  if (st.x.qubit || st.scratch_x < 0 || st.kb < 4 || st.nb > 4 || st.mb < 8 ||
      st.mb + st.kb > dev::kGatherMaxBits || st.x_in.size() < 2)
    return;
  const std::set<int> Ks(st.klab.begin(), st.klab.end());
  std::vector<int> kx;
  for (int l : st.x_in)
    if (Ks.count(l)) kx.push_back(l);
  if (kx != st.klab || !Ks.count(st.x_in.end()[-1]) || !Ks.count(st.x_in.end()[-2])) return;
  std::vector<int> xa = st.mlab;
  xa.insert(xa.end(), st.klab.begin(), st.klab.end());
  const PermDesc pd = make_perm_desc(st.x_in, xa);
  if (pd.perm[0] != 0 || pd.perm[1] != 1) return;
  ga = dev::SplitGather{};
  ga.nm = st.mb;
  ga.nk = st.kb - 2;
  for (int j = 0; j < ga.nk; ++j) ga.kpos[j] = (int8_t)pd.perm[2 + j];
  for (int j = 0; j < ga.nm; ++j) ga.mpos[j] = (int8_t)pd.perm[st.kb + j];
  use = 1;
}

void build_grid_device(qflex_grid* g, hipStream_t s) {
  for (CircuitState& cs : g->circ) {
    cs.tuned.assign(cs.plan.steps.size(), -1);
    cs.tuned_grad.assign(3 * cs.plan.steps.size(), -1);
  }
  std::vector<dev::GridPiece> pieces;
  std::vector<double2> mats;
  std::vector<int32_t> pos;
  std::vector<std::vector<dev::GridQubit>> qds(g->circ.size());
  std::vector<uint32_t> bidx;
  std::vector<int> max_nlb(g->circ.size(), 0);
  int64_t total = 0;
  for (size_t ci = 0; ci < g->circ.size(); ++ci) {
    CircuitState& cs = g->circ[ci];
    const Model& m = cs.model;
    const Plan& P = cs.plan;
    cs.grid_offset = total;
    cs.qubit_offset.assign(m.n, 0);
    const int mat_base = (int)(mats.size() / 4);
    cs.mat_base = mat_base;
    for (const cdouble& z : m.mats) mats.push_back(make_double2(z.real(), z.imag()));
    int64_t off = 0;
    for (int q = 0; q < m.n; ++q) {
      const QubitLayout& L = P.qubits[q];
      const int nb = (int)L.storage.size();
      cs.qubit_offset[q] = off;
      dev::GridQubit d{};
      d.offset = total + off;
      off += int64_t(1) << nb;
      off = (off + 63) & ~int64_t(63);  // keep every tensor 512-byte aligned
      auto where = [&](int label) {
        const int i = int(std::find(L.storage.begin(), L.storage.end(), label) - L.storage.begin());
        if (i >= nb) fail(QFLEX_E_DEVICE, "internal: label missing from a qubit layout");
        return nb - 1 - i;
      };
      d.pos_out = where(P.out_label(q));
      d.pos_base = (int)pos.size();
      int nlb = 0;
      std::vector<int> link_start(m.links.size(), 0);
      for (int l : m.qlinks[q]) {
        link_start[l] = nlb;
        for (int j = 0; j < m.links[l].bits; ++j) pos.push_back(where(P.link_base[l] + j));
        nlb += m.links[l].bits;
      }
      d.nlb = nlb;
      max_nlb[ci] = std::max(max_nlb[ci], nlb);
      d.piece_begin = (int)pieces.size();
      for (const Piece& pc : m.timeline[q]) {
        dev::GridPiece gp{};
        gp.mat = mat_base + pc.mat;
        if (pc.link >= 0) {
          gp.kshift = nlb - (link_start[pc.link] + pc.koff + pc.kbits);
          gp.kmask = (1 << pc.kbits) - 1;
        }
        pieces.push_back(gp);
      }
      d.piece_end = (int)pieces.size();
      qds[ci].push_back(d);
    }
    total += off;
    cs.bidx_offset = (int64_t)bidx.size();
    bidx.insert(bidx.end(), P.batch_index.begin(), P.batch_index.end());
  }
  g->grid_elems = total;
  QHIP(hipMalloc(&g->grid, sizeof(float2) * std::max<int64_t>(total, 1)));
  QHIP(hipMalloc(&g->bidx, sizeof(uint32_t) * std::max<size_t>(bidx.size(), 1)));
  DevBuf& dq = g->gq;
  DevBuf& dp = g->gpieces;
  DevBuf& dm = g->gmats;
  DevBuf& dpos = g->gpos;
  size_t nq = 0;
  for (auto& v : qds) nq += v.size();
  std::vector<dev::GridQubit> allq;
  for (size_t ci = 0; ci < qds.size(); ++ci) {
    g->circ[ci].qdesc_base = (int64_t)allq.size();
    g->circ[ci].max_nlb = max_nlb[ci];
    for (auto& d : qds[ci]) g->max_pieces = std::max(g->max_pieces, d.piece_end - d.piece_begin);
    allq.insert(allq.end(), qds[ci].begin(), qds[ci].end());
  }
  g->n_mats = (int64_t)(mats.size() / 4);
  try {
    dq.reserve(sizeof(dev::GridQubit) * std::max<size_t>(nq, 1));
    dp.reserve(sizeof(dev::GridPiece) * std::max<size_t>(pieces.size(), 1));
    dm.reserve(sizeof(double2) * std::max<size_t>(mats.size(), 1));
    dpos.reserve(sizeof(int32_t) * std::max<size_t>(pos.size(), 1));
    QHIP(hipMemcpyAsync(dq.p, allq.data(), sizeof(dev::GridQubit) * nq, hipMemcpyHostToDevice, s));
    QHIP(hipMemcpyAsync(dp.p, pieces.data(), sizeof(dev::GridPiece) * pieces.size(),
                        hipMemcpyHostToDevice, s));
    QHIP(hipMemcpyAsync(dm.p, mats.data(), sizeof(double2) * mats.size(), hipMemcpyHostToDevice, s));
    QHIP(hipMemcpyAsync(dpos.p, pos.data(), sizeof(int32_t) * pos.size(), hipMemcpyHostToDevice, s));
    if (!bidx.empty())
      QHIP(hipMemcpyAsync(g->bidx, bidx.data(), sizeof(uint32_t) * bidx.size(),
                          hipMemcpyHostToDevice, s));
    size_t qbase = 0;
    for (size_t ci = 0; ci < g->circ.size(); ++ci) {
      const int n = (int)qds[ci].size();
      dev::grid_build(static_cast<const dev::GridQubit*>(dq.p) + qbase, n, max_nlb[ci],
                      static_cast<const dev::GridPiece*>(dp.p), static_cast<const double2*>(dm.p),
                      static_cast<const int32_t*>(dpos.p), g->grid, s);
      qbase += n;
    }
    QHIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    throw;
  }
  // permutation tiles of every step
  for (auto& cs : g->circ) {
    const size_t ns = cs.plan.steps.size();
    cs.px.assign(ns, dev::PermTile{});
    cs.py.assign(ns, dev::PermTile{});
    cs.gather_x.assign(ns, 0);  // the split set-up adds the gathered split products
    cs.gx.assign(ns, dev::SplitGather{});
    for (size_t i = 0; i < ns; ++i) {
      const Step& st = cs.plan.steps[i];
      if (st.scratch_x >= 0) cs.px[i] = dev::make_perm_tile(st.px.nbits, st.px.perm.data());
      if (st.scratch_y >= 0) cs.py[i] = dev::make_perm_tile(st.py.nbits, st.py.perm.data());
      c64_gather(st, cs.gx[i], cs.gather_x[i]);
    }
  }
  if (g->precision == QFLEX_PREC_SPLIT_BF16 || g->precision == QFLEX_PREC_SPLIT_FP16)
    prepare_split(g, s);
  prepare_fused(g, s);
}

// The fused programs of every circuit that fits (complex64 grids, fused option not -1),
// uploaded in one buffer.
void prepare_fused(qflex_grid* g, hipStream_t s) {
  for (CircuitState& cs : g->circ) cs.fused_ok = false;
  if (g->precision != QFLEX_PREC_C64 || g->fused_opt < 0) return;
  const size_t nc = g->circ.size();
  std::vector<FusedProgram> prog(nc);
  size_t bytes = 0;
  auto up16 = [](size_t b) { return (b + 15) & ~size_t(15); };
  for (size_t c = 0; c < nc; ++c) {
    CircuitState& cs = g->circ[c];
    const std::string why = build_fused_program(cs.plan, cs.model, prog[c]);
    if (!why.empty()) {
      if (g->fused_opt == 1)
        fail(QFLEX_E_INVALID, "fused contraction required, but circuit " + std::to_string(c) +
                                  " does not fit: " + why);
      continue;
    }
    cs.fused_ok = true;
    cs.fused = prog[c].header;
    cs.fused.bidx = g->bidx + cs.bidx_offset;
    for (int q = 0; q < cs.model.n; ++q)
      prog[c].qubits[q].grid_off = cs.grid_offset + cs.qubit_offset[q];
    bytes += up16(sizeof(dev::FusedStep) * prog[c].steps.size()) +
             up16(sizeof(dev::FusedQubit) * prog[c].qubits.size()) +
             up16(sizeof(uint16_t) * prog[c].tables.size());
  }
  if (bytes == 0) return;
  dev::fused_setup();
  g->fused_prog.reserve(bytes);
  std::vector<char> host(bytes);
  size_t at = 0;
  for (size_t c = 0; c < nc; ++c) {
    CircuitState& cs = g->circ[c];
    if (!cs.fused_ok) continue;
    char* base = static_cast<char*>(g->fused_prog.p);
    const size_t sb = sizeof(dev::FusedStep) * prog[c].steps.size();
    const size_t qb = sizeof(dev::FusedQubit) * prog[c].qubits.size();
    const size_t tb = sizeof(uint16_t) * prog[c].tables.size();
    std::memcpy(host.data() + at, prog[c].steps.data(), sb);
    cs.fused.steps = reinterpret_cast<const dev::FusedStep*>(base + at);
    at += up16(sb);
    std::memcpy(host.data() + at, prog[c].qubits.data(), qb);
    cs.fused.qubits = reinterpret_cast<const dev::FusedQubit*>(base + at);
    at += up16(qb);
    std::memcpy(host.data() + at, prog[c].tables.data(), tb);
    cs.fused.tables = reinterpret_cast<const uint16_t*>(base + at);
    at += up16(tb);
  }
  QHIP(hipMemcpyAsync(g->fused_prog.p, host.data(), bytes, hipMemcpyHostToDevice, s));
  QHIP(hipStreamSynchronize(s));
}

// Tag for the next absmax() (or product maximum) into the fp16 scale slots: tags grow, so a
// slot never needs clearing; when they would wrap, every slot that calls rewrite is cleared
// and the tags start again (the qubit slots are written once, at build, and only read after).
static uint32_t next_amax_tag(qflex_grid* g, hipStream_t s) {
  if (g->amax_tag == UINT32_MAX) {  // clear every slot that calls rewrite
    dev::fill_zero(reinterpret_cast<double*>(g->amax), 2, s);
    for (const CircuitState& cs : g->circ)
      for (int64_t sl : cs.xcache_slot)
        if (sl >= 0) dev::fill_zero(reinterpret_cast<double*>(g->amax + sl), 1, s);
    if (g->node_amax) dev::fill_zero(reinterpret_cast<double*>(g->node_amax), g->n_node_amax, s);
    g->amax_tag = 0;
    g->resume.valid = false;  // their scales are gone: nothing is reused across this point
  }
  return ++g->amax_tag;
}

// Split-precision set-up: choose the steps that run as 16-bit products, pre-split the qubit
// tensors they read (A layout for a row operand, B layout for a column operand; the fixed
// leading bits stay leading so that bit-string and cut offsets only scale), and build the
// permute+split descriptors of intermediate operands.
void prepare_split(qflex_grid* g, hipStream_t s) {
  const bool f16 = g->precision == QFLEX_PREC_SPLIT_FP16;
  int64_t total = 0;
  int64_t n_slots = 2;
  int64_t n_node_slots = 0;
  struct Job {
    int circuit;
    int64_t src, dst;
    int nfixed, nbits, kbits;
    bool role_b;
    PermDesc pd;
    int64_t slot;
  };
  std::vector<Job> jobs;
  for (auto& cs : g->circ) {
    const Plan& P = cs.plan;
    const size_t ns = P.steps.size();
    cs.split.assign(ns, 0);
    cs.sx.assign(ns, dev::PermTile{});
    cs.sy.assign(ns, dev::PermTile{});
    cs.gather_y.assign(ns, 0);
    cs.gy.assign(ns, dev::SplitGather{});
    cs.xcache_offset.assign(ns, -1);
    cs.xcache_slot.assign(ns, -1);
    cs.xcache_elems = 0;
    cs.node_slot.assign(P.nodes.size(), -1);
    cs.qsplit_offset.assign(cs.model.n, -1);
    cs.qamax_slot.assign(cs.model.n, -1);
    cs.split_a_elems = cs.split_b_elems = 0;
    for (size_t i = 0; i < ns; ++i) {
      const Step& st = P.steps[i];
      const int64_t M = int64_t(1) << st.mb, N = int64_t(1) << st.nb, K = int64_t(1) << st.kb;
      if (!dev::gemm_split_ok(M, N, K)) continue;
      cs.split[i] = 1;
      if (f16) cs.node_slot[st.out] = n_node_slots++;
      // The order of the contracted labels is this step's own choice.  For an intermediate
      // x, order them as x stores them: when x's 2 lowest storage labels are contracted ones,
      // every group of 4 consecutive k is then 32 contiguous bytes of x, and the product reads
      // x straight from its complex64 storage (no permutation or split pass over x).
      std::vector<int> klab = st.klab;
      bool gather = false;
      // an intermediate x that outlives this step's slices (it depends on fewer cuts) is split
      // once per recomputation into a cache instead of being gathered every time
      const bool cached = !st.x.qubit && P.nodes[st.x.id].deps != st.deps;
      if (cached) {
        cs.xcache_offset[i] = cs.xcache_elems;
        cs.xcache_elems +=
            ((int64_t(dev::kSplitValues) << P.nodes[st.x.id].labels.size()) + 63) & ~int64_t(63);
        if (f16) cs.xcache_slot[i] = n_slots++;
      }
      if (!cached && !st.x.qubit && st.kb >= 4 && st.x_in.size() >= 2) {
        const std::set<int> K(st.klab.begin(), st.klab.end());
        if (K.count(st.x_in.end()[-1]) && K.count(st.x_in.end()[-2])) {
          klab.clear();
          for (int l : st.x_in)
            if (K.count(l)) klab.push_back(l);
          gather = true;
        }
      }
      // Failing that, the same for an intermediate y: its contracted labels ordered as y stores
      // them, which x (from a cache, a qubit tensor's split or a permutation) then follows.
      bool gather_y = false;
      if (!gather && !st.y.qubit && st.kb >= 4 && st.y_in.size() >= 2) {
        const std::set<int> K(st.klab.begin(), st.klab.end());
        if (K.count(st.y_in.end()[-1]) && K.count(st.y_in.end()[-2])) {
          klab.clear();
          for (int l : st.y_in)
            if (K.count(l)) klab.push_back(l);
          gather_y = true;
        }
      }
      const std::vector<int> xa = [&] { auto v = st.mlab; v.insert(v.end(), klab.begin(), klab.end()); return v; }();
      const std::vector<int> yb = [&] { auto v = st.nlab; v.insert(v.end(), klab.begin(), klab.end()); return v; }();
      if (gather) {
        const PermDesc pd = make_perm_desc(st.x_in, xa);
        dev::SplitGather& ga = cs.gx[i];
        ga.nm = st.mb;
        ga.nk = st.kb - 2;
        bool ok = st.mb + st.kb <= dev::kGatherMaxBits;
        for (int j = 0; j < 2 && ok; ++j) ok = pd.perm[j] == j;
        for (int j = 0; ok && j < ga.nk; ++j) ga.kpos[j] = (int8_t)pd.perm[2 + j];
        for (int j = 0; ok && j < ga.nm; ++j) ga.mpos[j] = (int8_t)pd.perm[st.kb + j];
        cs.gather_x[i] = ok;
      }
      if (gather_y) {
        const PermDesc pd = make_perm_desc(st.y_in, yb);
        dev::SplitGather& gb = cs.gy[i];
        gb.nm = st.nb;
        gb.nk = st.kb - 2;
        bool ok = st.nb + st.kb <= dev::kGatherMaxBits;
        for (int j = 0; j < 2 && ok; ++j) ok = pd.perm[j] == j;
        for (int j = 0; ok && j < gb.nk; ++j) gb.kpos[j] = (int8_t)pd.perm[2 + j];
        for (int j = 0; ok && j < gb.nm; ++j) gb.mpos[j] = (int8_t)pd.perm[st.kb + j];
        cs.gather_y[i] = ok;
      }
      for (int side = 0; side < 2; ++side) {
        const Operand& o = side ? st.y : st.x;
        const std::vector<int>& in = side ? st.y_in : st.x_in;
        const std::vector<int>& want = side ? yb : xa;
        const PermDesc pd = make_perm_desc(in, want);
        if (o.qubit) {
          const QubitLayout& L = P.qubits[o.id];
          Job j{(int)(&cs - &g->circ[0]), cs.grid_offset + cs.qubit_offset[o.id], total,
                L.n_fixed, L.free_bits(), st.kb, side == 1, pd, f16 ? n_slots : -1};
          if (f16) cs.qamax_slot[o.id] = n_slots++;
          cs.qsplit_offset[o.id] = total;
          total += ((int64_t(dev::kSplitValues) << L.storage.size()) + 63) & ~int64_t(63);
          jobs.push_back(j);
        } else if (side == 0 && cached) {
          cs.sx[i] = dev::make_perm_tile(pd.nbits, pd.perm.data());
        } else {  // also for a gathered x: the autotuner may prefer permuting it
          (side ? cs.sy[i] : cs.sx[i]) = dev::make_perm_tile(pd.nbits, pd.perm.data());
          const int64_t e = int64_t(dev::kSplitValues) << P.nodes[o.id].labels.size();
          if (side) cs.split_b_elems = std::max(cs.split_b_elems, e);
          else cs.split_a_elems = std::max(cs.split_a_elems, e);
        }
      }
    }
  }
  if (f16) {
    QHIP(hipMalloc(&g->amax, sizeof(uint64_t) * n_slots));
    g->n_amax = n_slots;
    g->amax_tag = 0;
    dev::fill_zero(reinterpret_cast<double*>(g->amax), n_slots, s);
    if (n_node_slots) {
      QHIP(hipMalloc(&g->node_amax, sizeof(uint64_t) * n_node_slots));
      g->n_node_amax = n_node_slots;
      dev::fill_zero(reinterpret_cast<double*>(g->node_amax), n_node_slots, s);
    }
  }
  g->qsplit_jobs.clear();
  if (total == 0) return;
  QHIP(hipMalloc(&g->grid_split, sizeof(uint16_t) * total));
  for (const Job& j : jobs) {
    QubitSplitJob q;
    q.circuit = j.circuit;
    q.src = j.src;
    q.dst = j.dst;
    q.nfixed = j.nfixed;
    q.nbits = j.nbits;
    q.kbits = j.kbits;
    q.tile = dev::make_perm_tile(j.nbits, j.pd.perm.data());
    q.slot = j.slot;
    g->qsplit_jobs.push_back(q);
  }
  split_qubits(g, -1, s);
  QHIP(hipStreamSynchronize(s));
}

// Pre-split the qubit tensors of circuit c (every circuit for c < 0) for 16-bit products.
void split_qubits(qflex_grid* g, int c, hipStream_t s) {
  for (const QubitSplitJob& j : g->qsplit_jobs) {
    if (c >= 0 && j.circuit != c) continue;
    const int64_t n = int64_t(1) << (j.nfixed + j.nbits);
    uint64_t* slot = j.slot >= 0 ? g->amax + j.slot : nullptr;
    // one scale per qubit tensor, over every value of its fixed (bit-string / cut) indexes;
    // the slot is cleared first, since its previous tag may exceed the next one after a wrap
    if (slot) {
      dev::fill_zero(reinterpret_cast<double*>(slot), 1, s);
      dev::absmax(g->grid + j.src, n, slot, next_amax_tag(g, s), s);
    }
    dev::split_permute(g->grid + j.src, g->grid_split + j.dst, int64_t(1) << j.nfixed, j.tile,
                       j.kbits, slot, s);
  }
}

void update_gates(qflex_grid* g, int c, const qflex_circuit& circuit, hipStream_t s) {
  if (c < 0 || c >= (int)g->circ.size()) fail(QFLEX_E_INVALID, "bad circuit index");
  CircuitState& cs = g->circ[c];
  Model m = build_model(circuit);
  const Model& o = cs.model;
  // the plan, the tensor layouts and the piece tables hold as long as the structure does
  bool same = m.n == o.n && m.xy == o.xy && m.gates.size() == o.gates.size() &&
              m.links.size() == o.links.size() && m.mats.size() == o.mats.size() &&
              m.timeline.size() == o.timeline.size();
  for (size_t i = 0; same && i < m.gates.size(); ++i) {
    const Gate &a = m.gates[i], &b = o.gates[i];
    same = a.cycle == b.cycle && a.kind == b.kind && a.q0 == b.q0 && a.q1 == b.q1;
  }
  for (size_t l = 0; same && l < m.links.size(); ++l)
    same = m.links[l].lo == o.links[l].lo && m.links[l].hi == o.links[l].hi &&
           m.links[l].gate_ids == o.links[l].gate_ids && m.links[l].rank == o.links[l].rank;
  for (size_t q = 0; same && q < m.timeline.size(); ++q) {
    same = m.timeline[q].size() == o.timeline[q].size();
    for (size_t i = 0; same && i < m.timeline[q].size(); ++i) {
      const Piece &a = m.timeline[q][i], &b = o.timeline[q][i];
      same = a.gate == b.gate && a.link == b.link && a.kbits == b.kbits && a.koff == b.koff &&
             a.mat == b.mat && a.hi_side == b.hi_side;
    }
  }
  if (!same)
    fail(QFLEX_E_INVALID, "the updated circuit differs in structure (qubits, couplers, cycles, "
                          "kinds or bond ranks); build a new grid for it");
  std::vector<double2> mats;
  for (const cdouble& z : m.mats) mats.push_back(make_double2(z.real(), z.imag()));
  // nothing kept from earlier calls depends on the old tensors after this
  g->resume.valid = false;
  QHIP(hipMemcpyAsync(static_cast<double2*>(g->gmats.p) + 4 * (int64_t)cs.mat_base, mats.data(),
                      sizeof(double2) * mats.size(), hipMemcpyHostToDevice, s));
  dev::grid_build(static_cast<const dev::GridQubit*>(g->gq.p) + cs.qdesc_base, m.n, cs.max_nlb,
                  static_cast<const dev::GridPiece*>(g->gpieces.p),
                  static_cast<const double2*>(g->gmats.p), static_cast<const int32_t*>(g->gpos.p),
                  g->grid, s);
  if (g->grid_split) split_qubits(g, c, s);
  cs.model = std::move(m);
  QHIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------------ autotuning
float time_launches(qflex_grid* g, hipStream_t s, const std::function<void()>& launch) {
  if (!g->tune_ev[0]) {
    QHIP(hipEventCreate(&g->tune_ev[0]));
    QHIP(hipEventCreate(&g->tune_ev[1]));
  }
  const bool on = g->prof.on;
  g->prof.on = false;
  ++g->n_tuned;
  launch();  // warm-up
  // the best of three timed runs: a single run's time varies with the clock and with other
  // work in flight, which made the choices differ between otherwise identical grids
  float best = 0;
  for (int rep = 0; rep < 3; ++rep) {
    QHIP(hipEventRecord(g->tune_ev[0], s));
    launch();
    QHIP(hipEventRecord(g->tune_ev[1], s));
    QHIP(hipEventSynchronize(g->tune_ev[1]));
    float ms = 0;
    QHIP(hipEventElapsedTime(&ms, g->tune_ev[0], g->tune_ev[1]));
    if (rep == 0 || ms < best) best = ms;
  }
  g->prof.on = on;
  return best;
}

int tune_gemm(qflex_grid* g, hipStream_t s, const dev::Gemm& gm) {
  // a choice made before for this device and shape (this process, or a loaded cache file)
  const std::string key = g->device_sig + "|c64|" + std::to_string(gm.M) + "x" +
                          std::to_string(gm.N) + "x" + std::to_string(gm.K) + "|t" +
                          std::to_string(gm.ta) + std::to_string(gm.tb) + "|b" +
                          std::to_string(gm.batch) + "|ws" + std::to_string(gm.ws ? 1 : 0);
  int best_v = -1;
  if (tune_cache_get(key, &best_v) && best_v < dev::kGemmVariants &&
      dev::gemm_variant_fits(gm, best_v))
    return best_v;
  best_v = -1;
  float best = 0;
  for (int v = 0; v < dev::kGemmVariants; ++v) {
    if (!dev::gemm_variant_fits(gm, v)) continue;
    dev::Gemm t = gm;
    t.force_variant = v;
    const float ms = time_launches(g, s, [&] { dev::gemm(t, s); });
    if (best_v < 0 || ms < best) best_v = v, best = ms;
  }
  if (best_v >= 0) tune_cache_put(key, best_v);
  return best_v;
}

// ------------------------------------------------------------------------------ slices
std::vector<int64_t> select_slices(int64_t total, double fidelity, uint64_t seed, int mode) {
  if (!(fidelity > 0.0 && fidelity <= 1.0)) fail(QFLEX_E_INVALID, "fidelity must be in (0, 1]");
  if (mode != QFLEX_SLICES_RANDOM && mode != QFLEX_SLICES_BLOCK)
    fail(QFLEX_E_INVALID, "unknown slice_mode");
  const double k = fidelity * (double)total;
  const double kr = std::round(k);
  if (std::fabs(k - kr) > 1e-9 * std::max(1.0, k) || kr < 1)
    fail(QFLEX_E_PLAN, "fidelity * slices must be an integer >= 1");
  uint64_t state = seed;
  auto next = [&]() {  // SplitMix64
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  if (mode == QFLEX_SLICES_BLOCK) {  // k consecutive ids from a seeded multiple of k
    const int64_t kk = (int64_t)kr;
    if (total % kk) fail(QFLEX_E_PLAN, "block slice subsets need fidelity * slices to divide them");
    const int64_t j = (int64_t)(next() % (uint64_t)(total / kk));
    std::vector<int64_t> b(kk);
    std::iota(b.begin(), b.end(), j * kk);
    return b;
  }
  std::vector<int64_t> a(total);
  std::iota(a.begin(), a.end(), 0);
  for (int64_t i = total - 1; i > 0; --i) {
    const int64_t j = (int64_t)(next() % (uint64_t)(i + 1));
    std::swap(a[i], a[j]);
  }
  a.resize((size_t)kr);
  std::sort(a.begin(), a.end());
  return a;
}

// ------------------------------------------------------------------------------ contract
namespace {

struct View {
  const float2* base = nullptr;
  const int64_t* off = nullptr;
  int64_t bs = 0, add = 0;
};

}  // namespace

std::vector<std::vector<int64_t>> prepare_call(qflex_grid* g, const uint8_t* bits,
                                               const int64_t* bs_offsets, double fidelity,
                                               uint64_t seed, const int64_t* slice_ids,
                                               const int64_t* slice_offsets, const void* amps,
                                               hipStream_t s, bool pinned_ok) {
  const int nc = (int)g->circ.size();
  // ---- validation (host only)
  if (!bs_offsets) fail(QFLEX_E_INVALID, "NULL argument");
  if (bs_offsets[0] != 0) fail(QFLEX_E_INVALID, "bs_offsets[0] must be 0");
  if (bs_offsets[nc] > 0 && (!bits || !amps)) fail(QFLEX_E_INVALID, "NULL argument");
  std::vector<int64_t> byte_off(nc + 1, 0);
  for (int c = 0; c < nc; ++c) {
    if (bs_offsets[c + 1] < bs_offsets[c]) fail(QFLEX_E_INVALID, "bs_offsets must not decrease");
    byte_off[c + 1] = byte_off[c] + (bs_offsets[c + 1] - bs_offsets[c]) * g->circ[c].model.n;
  }
  for (int64_t i = 0; i < byte_off[nc]; ++i)
    if (bits[i] > 1) fail(QFLEX_E_INVALID, "bit-string entries must be 0 or 1");
  std::vector<std::vector<int64_t>> sel(nc);
  for (int c = 0; c < nc; ++c) {
    const int64_t S = g->circ[c].plan.num_slices();
    if (slice_ids) {
      if (!slice_offsets) fail(QFLEX_E_INVALID, "slice_ids given without slice_offsets");
      if (slice_offsets[c + 1] < slice_offsets[c] || (c == 0 && slice_offsets[0] != 0))
        fail(QFLEX_E_INVALID, "bad slice_offsets");
      sel[c].assign(slice_ids + slice_offsets[c], slice_ids + slice_offsets[c + 1]);
      std::sort(sel[c].begin(), sel[c].end());
      for (size_t i = 0; i < sel[c].size(); ++i) {
        if (sel[c][i] < 0 || sel[c][i] >= S) fail(QFLEX_E_INVALID, "slice id out of range");
        if (i && sel[c][i] == sel[c][i - 1]) fail(QFLEX_E_INVALID, "slice id repeated");
      }
    } else {
      sel[c] = select_slices(S, fidelity, seed, g->slice_mode);
    }
  }
  QHIP(hipGetLastError());
  // ---- per-bit-string output offsets of every closed qubit tensor, all circuits
  std::vector<int64_t> offs_base(nc + 1, 0);
  for (int c = 0; c < nc; ++c)
    offs_base[c + 1] = offs_base[c] + (bs_offsets[c + 1] - bs_offsets[c]) * g->circ[c].model.n;
  const size_t offs_bytes = sizeof(int64_t) * std::max<int64_t>(offs_base[nc], 1);
  // a call whose circuits all run the fused kernel reads the table in place from pinned host
  // memory: each kernel reads its bit-string's entries once, and no copy precedes it
  bool pinned = pinned_ok;
  for (int c = 0; c < nc; ++c) pinned = pinned && g->circ[c].fused_ok && !sel[c].empty();
  int64_t* oh = nullptr;
  g->offs_pinned_slot = -1;
  if (pinned) {
    const int k = g->offs_pinned_next;
    g->offs_pinned_next ^= 1;
    // the call before last read this buffer: wait for its launches before rewriting it
    if (g->offs_pinned_done[k]) QHIP(hipEventSynchronize(g->offs_pinned_done[k]));
    else QHIP(hipEventCreateWithFlags(&g->offs_pinned_done[k], hipEventDisableTiming));
    g->offs_pinned[k].reserve(offs_bytes);
    if (g->offs_pinned_at[k] != g->offs_pinned[k].p) {
      QHIP(hipHostGetDevicePointer(&g->offs_pinned_dev[k], g->offs_pinned[k].p, 0));
      g->offs_pinned_at[k] = g->offs_pinned[k].p;
    }
    oh = static_cast<int64_t*>(g->offs_pinned[k].p);
    g->offs_cur = static_cast<const int64_t*>(g->offs_pinned_dev[k]);
    g->offs_pinned_slot = k;
  } else {
    if (g->offs_done) QHIP(hipEventSynchronize(g->offs_done));
    g->offs_host.reserve(offs_bytes);
    g->offs.reserve(offs_bytes);
    oh = static_cast<int64_t*>(g->offs_host.p);
    g->offs_cur = static_cast<const int64_t*>(g->offs.p);
  }
  for (int c = 0; c < nc; ++c) {
    const CircuitState& cs = g->circ[c];
    const int n = cs.model.n;
    const int64_t nbs = bs_offsets[c + 1] - bs_offsets[c];
    for (int q = 0; q < n; ++q) {
      const int sh = cs.plan.qubits[q].out_shift;
      for (int64_t b = 0; b < nbs; ++b)
        oh[offs_base[c] + q * nbs + b] =
            sh < 0 ? 0 : (int64_t)bits[byte_off[c] + b * n + q] << sh;
    }
  }
  if (!pinned) {
    QHIP(hipMemcpyAsync(g->offs.p, oh, offs_bytes, hipMemcpyHostToDevice, s));
    if (!g->offs_done) QHIP(hipEventCreateWithFlags(&g->offs_done, hipEventDisableTiming));
    QHIP(hipEventRecord(g->offs_done, s));
  }
  return sel;
}

void contract(qflex_grid* g, const uint8_t* bits, const int64_t* bs_offsets, double fidelity,
              uint64_t seed, const int64_t* slice_ids, const int64_t* slice_offsets,
              double* amps, int32_t out_flags, hipStream_t s_user) {
  hipStream_t s = s_user;
  const int nc = (int)g->circ.size();
  if (out_flags != QFLEX_OUT_HOST && out_flags != QFLEX_OUT_DEVICE &&
      out_flags != (QFLEX_OUT_DEVICE | QFLEX_OUT_ACCUMULATE))
    fail(QFLEX_E_INVALID, "amps_on_device must be 0, 1 or 3 (accumulating needs device output)");
  const bool amps_on_device = (out_flags & QFLEX_OUT_DEVICE) != 0;
  const bool accumulate = (out_flags & QFLEX_OUT_ACCUMULATE) != 0;
  const std::vector<std::vector<int64_t>> sel = prepare_call(
      g, bits, bs_offsets, fidelity, seed, slice_ids, slice_offsets, amps, s, true);
  // the pinned offsets buffer this call's kernels read in place, if any: its event is
  // recorded after them, also when a launch fails part-way
  struct PinnedRelease {
    qflex_grid* g;
    hipStream_t s;
    ~PinnedRelease() {
      if (g->offs_pinned_slot >= 0)
        (void)hipEventRecord(g->offs_pinned_done[g->offs_pinned_slot], s);
      g->offs_pinned_slot = -1;
    }
  } pinned_release{g, s};
  qflex_stats st{};
  const int64_t tuned0 = g->n_tuned;
  std::vector<int64_t> offs_base(nc + 1, 0);
  for (int c = 0; c < nc; ++c)
    offs_base[c + 1] = offs_base[c] + (bs_offsets[c + 1] - bs_offsets[c]) * g->circ[c].model.n;
  const int64_t* offs_dev = g->offs_cur;

  // every circuit runs the fused small-plan kernel (a circuit with no slice selected would
  // launch nothing)
  bool all_fused = true;
  for (int c = 0; c < nc; ++c)
    all_fused = all_fused && g->circ[c].fused_ok && !sel[c].empty();
  // graph mode (below) captures and replays the call's launches; a call whose circuits are all
  // fused is launched directly: one kernel per circuit and 64 slices, which a graph would not
  // shorten (its own launch costs more than the launches it saves)
  const bool graph = g->graph_mode && !all_fused;
  // free device memory sizes the step path's batches of bit-strings (fused circuits take
  // every bit-string in one launch and no arena)
  size_t free_b = 0, total_b = 0;
  bool need_free = false;
  for (int c = 0; c < nc; ++c) need_free = need_free || !g->circ[c].fused_ok;
  if (need_free && g->bitstring_batch <= 0) QHIP(hipMemGetInfo(&free_b, &total_b));
  // ---- batch of bit-strings contracted together, per circuit; one arena for the largest
  std::vector<int64_t> batch(nc, 1);
  size_t arena_need = sizeof(float2);
  int64_t amp_total = 0;
  for (int c = 0; c < nc; ++c) {
    const Plan& P = g->circ[c].plan;
    const int64_t nbs = bs_offsets[c + 1] - bs_offsets[c];
    amp_total += nbs * (int64_t(1) << P.open.size());
    if (g->circ[c].fused_ok) continue;
    int64_t B = g->bitstring_batch > 0 ? g->bitstring_batch : 0;
    if (B == 0) {
      const double per = 8.0 * (double)std::max<int64_t>(P.arena_elems, 1);
      const double budget = std::min(0.5 * ((double)free_b + (double)g->arena.bytes),
                                     96.0 * (1ull << 30));
      B = (int64_t)std::max(1.0, std::floor(budget / per));
      B = std::min<int64_t>(B, 256);
    }
    B = std::min<int64_t>(std::max<int64_t>(B, 1), std::max<int64_t>(nbs, 1));
    B = std::min<int64_t>(B, 65535);
    batch[c] = B;
    arena_need = std::max(arena_need, sizeof(float2) * (size_t)(P.arena_elems * B));
  }
  g->arena.reserve(arena_need);
  size_t split_need = 0;
  for (int c = 0; c < nc; ++c)
    split_need = std::max(split_need, sizeof(uint16_t) * (size_t)batch[c] *
                                          (size_t)(g->circ[c].split_a_elems +
                                                   g->circ[c].split_b_elems));
  if (split_need) g->split_scratch.reserve(split_need);
  size_t cache_need = 0;
  for (int c = 0; c < nc; ++c)
    cache_need = std::max(cache_need, sizeof(uint16_t) * (size_t)batch[c] *
                                          (size_t)g->circ[c].xcache_elems);
  if (cache_need) g->split_cache.reserve(cache_need);
  // slice sums go straight into the caller's buffer when the call accumulates into it, or
  // when it is device memory and no graph is captured (a graph keeps the grid's own buffer,
  // so that a replay does not depend on the caller's output address)
  const bool direct = accumulate || (amps_on_device && !graph);
  if (!direct) g->amps64.reserve(sizeof(double2) * std::max<int64_t>(amp_total, 1));
  float2* arena = static_cast<float2*>(g->arena.p);
  double2* acc_all = direct ? reinterpret_cast<double2*>(amps)
                            : static_cast<double2*>(g->amps64.p);
  // intermediates of the previous call's last batch stay usable unless a buffer moved; every
  // path below that does not finish invalidates them
  Resume& rs = g->resume;
  if (rs.valid && (rs.arena != g->arena.p || rs.cache != g->split_cache.p)) rs.valid = false;
  const Resume kept = rs;
  rs.valid = false;
  auto time_launches = [&](const std::function<void()>& launch) {
    return qflex::time_launches(g, s, launch);
  };
  bool tuning_pending = false;
  if (g->autotune)
    for (const CircuitState& cs : g->circ)
      if (!cs.fused_ok)  // the fused kernel has no variants to time
        for (int v : cs.tuned) tuning_pending = tuning_pending || v < 0;
  std::string key;
  bool capturing = false;
  const bool prof_was_on = g->prof.on;
  if (graph) {
    // capture and replay on the caller's stream; the null stream cannot capture, so then the
    // launches go to the grid's own stream, ordered after the caller's earlier work
    if (!s_user) {
      if (!g->graph_stream) {
        QHIP(hipStreamCreateWithFlags(&g->graph_stream, hipStreamNonBlocking));
        QHIP(hipEventCreateWithFlags(&g->graph_in, hipEventDisableTiming));
        QHIP(hipEventCreateWithFlags(&g->graph_out, hipEventDisableTiming));
      }
      QHIP(hipEventRecord(g->graph_in, s_user));
      QHIP(hipStreamWaitEvent(g->graph_stream, g->graph_in, 0));
      s = g->graph_stream;
    }
    key.reserve(256);
    const void* keyed[] = {g->arena.p, g->split_scratch.p, g->split_cache.p, acc_all,
                           g->offs.p, g->splitk_ws.p, s};
    for (const void* p : keyed)
      key += std::to_string(reinterpret_cast<uintptr_t>(p)) + ",";
    key += accumulate ? "+" : "=";
    for (int c = 0; c < nc; ++c) {
      key += "|" + std::to_string(bs_offsets[c + 1] - bs_offsets[c]) + ":" +
             std::to_string(batch[c]) + ":";
      for (int64_t id : sel[c]) key += std::to_string(id) + ",";
    }
    if (g->graph_exec && key == g->graph_key) {
      QHIP(hipGraphLaunch(g->graph_exec, s));
      st = g->graph_stats;
    } else if (tuning_pending) {
      // autotuning synchronises: this call runs eagerly, a later identical one is captured
    } else {
      if (g->graph_exec) {
        QHIP(hipGraphExecDestroy(g->graph_exec));
        g->graph_exec = nullptr;
        g->graph_key.clear();
      }
      g->prof.on = false;  // no event records inside a graph
      QHIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      capturing = true;
    }
  }
  auto end_capture = [&](bool launch) {
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &gr);
    capturing = false;
    g->prof.on = prof_was_on;
    if (e != hipSuccess || !gr) {
      if (gr) (void)hipGraphDestroy(gr);
      if (launch) fail(QFLEX_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      return;
    }
    if (!launch) {
      (void)hipGraphDestroy(gr);
      return;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess) fail(QFLEX_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    g->graph_exec = ex;
    g->graph_key = key;
    QHIP(hipGraphLaunch(ex, s));
  };
  const bool replayed = graph && !capturing && !tuning_pending;
  // every launch of this call (skipped when the graph replays them)
  auto enqueue = [&] {
    if (graph && g->amax) {
      // fp16 scale slots rewritten by every call start from zero in each replay (the tags of
      // their atomic maxima are fixed in the graph)
      dev::fill_zero(reinterpret_cast<double*>(g->amax), 2, s);
      for (const CircuitState& cs : g->circ)
        for (int64_t sl : cs.xcache_slot)
          if (sl >= 0) dev::fill_zero(reinterpret_cast<double*>(g->amax + sl), 1, s);
      if (g->node_amax) dev::fill_zero(reinterpret_cast<double*>(g->node_amax), g->n_node_amax, s);
    }
    // the sums start from zero, unless every circuit's fused kernel writes its own first
    if (!accumulate && !all_fused)
      dev::fill_zero(reinterpret_cast<double*>(acc_all), 2 * amp_total, s);
    bool first_batch = true;  // only the call's first batch can find its intermediates kept
    for (int c = 0; c < nc; ++c) {
      CircuitState& cs = g->circ[c];
      const Plan& P = cs.plan;
      const int64_t nbs = bs_offsets[c + 1] - bs_offsets[c];
      if (nbs == 0) continue;
      const int no = (int)P.open.size();
      const int64_t namp = int64_t(1) << no;
      const int64_t B = batch[c];
      double2* acc = acc_all + bs_offsets[c] * namp;
      const float2* grid = g->grid + cs.grid_offset;
      const auto& slices = sel[c];
      const int ncut = (int)P.cuts.size();
      if (cs.fused_ok) {
        // one workgroup per bit-string runs the whole plan (up to 64 slices per launch);
        // nothing stays in the arena for a later call
        double flops = 0;
        std::vector<int64_t> dg(ncut, -1), pv(ncut, -1);
        for (size_t si = 0; si < slices.size(); ++si) {
          int64_t rem = slices[si];
          uint32_t changed = 0;
          for (int ct = ncut - 1; ct >= 0; --ct) {
            dg[ct] = rem & ((int64_t(1) << P.cut_bits[ct]) - 1);
            rem >>= P.cut_bits[ct];
            if (dg[ct] != pv[ct]) changed |= 1u << ct;
          }
          pv = dg;
          for (const Step& stp : P.steps)
            if (si == 0 || (stp.deps & changed)) flops += stp.flops(), ++st.n_gemm;
        }
        g->prof.begin("fused_contract", flops * nbs, 8.0 * nbs * (double)P.arena_elems, s);
        dev::fused_contract(cs.fused, g->grid, offs_dev + offs_base[c], nbs, 0, nbs,
                            slices.data(), (int)slices.size(), acc, !accumulate && all_fused, s);
        g->prof.end(s);
        st.flops += flops * nbs;
        st.n_slices += (int64_t)slices.size();
        st.n_bitstrings += nbs;
        continue;
      }
      for (int64_t b0 = 0; b0 < nbs; b0 += B) {
        const int nb = (int)std::min<int64_t>(B, nbs - b0);
        std::vector<int64_t> digit(ncut, -1), prev(ncut, -1);
        // the batch's rows: circuit c's rows start after every earlier circuit's (each of
        // its own width n), which is where its offsets start too
        const uint8_t* batch_bits = bits + offs_base[c] + b0 * cs.model.n;
        const size_t batch_bytes = (size_t)nb * (size_t)cs.model.n;
        // resumed: the arena still holds this batch's intermediates for the cut values in prev
        const bool resumed = first_batch && !graph && kept.valid && kept.circuit == c &&
                             kept.batch == B && kept.bits.size() == batch_bytes &&
                             std::equal(kept.bits.begin(), kept.bits.end(), batch_bits);
        if (resumed) prev = kept.digits;
        first_batch = false;
        auto view = [&](const Operand& o) {
          View v;
          if (o.qubit) {
            const QubitLayout& L = P.qubits[o.id];
            v.base = grid + cs.qubit_offset[o.id];
            for (auto& cshift : L.cut_shift) v.add += digit[cshift.first] << cshift.second;
            if (L.out_shift >= 0) v.off = offs_dev + offs_base[c] + (int64_t)o.id * nbs + b0;
          } else {
            const Node& nd = P.nodes[o.id];
            v.base = arena + nd.offset * B;
            v.bs = nd.elems();
          }
          return v;
        };
        for (size_t si = 0; si < slices.size(); ++si) {
          int64_t rem = slices[si];
          for (int ct = ncut - 1; ct >= 0; --ct) {
            digit[ct] = rem & ((int64_t(1) << P.cut_bits[ct]) - 1);
            rem >>= P.cut_bits[ct];
          }
          uint32_t changed = 0;
          for (int ct = 0; ct < ncut; ++ct)
            if (digit[ct] != prev[ct]) changed |= 1u << ct;
          prev = digit;
          // every step runs for the first slice of a batch, unless the batch was resumed
          const bool fresh = si == 0 && !resumed;
          for (size_t k = 0; k < P.steps.size(); ++k) {
            const Step& stp = P.steps[k];
            if (!fresh && !(stp.deps & changed)) continue;
            View x = view(stp.x), y = view(stp.y);
            const bool is_split = !cs.split.empty() && cs.split[k];
            const int64_t M = int64_t(1) << stp.mb, N = int64_t(1) << stp.nb;
            const int64_t K = int64_t(1) << stp.kb;
            // one split product: gather (gather_y) = read x (y) straight from complex64 storage
            // (when the plan allows it), tile = output tile (-1: shape rule); `final` runs count
            // in stats
            auto run_split = [&](bool gather, bool gather_y, int tile, bool final) {
              uint16_t* sa = static_cast<uint16_t*>(g->split_scratch.p);
              uint16_t* sb = sa + B * cs.split_a_elems;
              dev::GemmSplit gs;
              gs.tile = tile;
              const bool f16 = g->amax != nullptr;
              // fp16 scales of intermediates that a split product produced (and measured)
              auto node_slot = [&](const Operand& o) -> uint64_t* {
                if (!f16 || o.qubit || cs.node_slot[o.id] < 0) return nullptr;
                return g->node_amax + cs.node_slot[o.id];
              };
              uint64_t* const xslot = node_slot(stp.x);
              uint64_t* const yslot = node_slot(stp.y);
              if (stp.x.qubit) {
                gs.A = g->grid_split + cs.qsplit_offset[stp.x.id];
                gs.a_add = x.add;
                gs.a_off = x.off;
                if (f16) gs.a_amax = g->amax + cs.qamax_slot[stp.x.id];
              } else if (cs.xcache_offset[k] >= 0) {
                uint16_t* xc = static_cast<uint16_t*>(g->split_cache.p) + B * cs.xcache_offset[k];
                if (f16) gs.a_amax = xslot ? xslot : g->amax + cs.xcache_slot[k];
                if (fresh || (P.nodes[stp.x.id].deps & changed)) {  // x was just recomputed
                  if (f16 && !xslot) {
                    g->prof.begin("absmax", 0, 8.0 * M * K * nb, s);
                    dev::absmax(x.base, M * K * nb, g->amax + cs.xcache_slot[k],
                                next_amax_tag(g, s), s);
                    g->prof.end(s);
                  }
                  g->prof.begin("split_permute", 0, 16.0 * M * K * nb, s);
                  dev::split_permute(x.base, xc, nb, cs.sx[k], stp.kb, gs.a_amax, s);
                  g->prof.end(s);
                  if (final) st.permute_bytes += 16.0 * M * K * nb, ++st.n_permute;
                }
                gs.A = xc;
                gs.a_bs = M * K;
              } else {
                if (f16 && xslot) {
                  gs.a_amax = xslot;
                } else if (f16) {
                  gs.a_amax = g->amax;
                  g->prof.begin("absmax", 0, 8.0 * M * K * nb, s);
                  dev::absmax(x.base, M * K * nb, g->amax, next_amax_tag(g, s), s);
                  g->prof.end(s);
                }
                if (gather) {
                  gs.Ac = x.base;
                  gs.a_bs = x.bs;
                  gs.ga = cs.gx[k];
                } else {
                  g->prof.begin("split_permute", 0, 16.0 * M * K * nb, s);
                  dev::split_permute(x.base, sa, nb, cs.sx[k], stp.kb, gs.a_amax, s);
                  g->prof.end(s);
                  if (final) st.permute_bytes += 16.0 * M * K * nb, ++st.n_permute;
                  gs.A = sa;
                  gs.a_bs = M * K;
                }
              }
              if (stp.y.qubit) {
                gs.B = g->grid_split + cs.qsplit_offset[stp.y.id];
                gs.b_add = y.add;
                gs.b_off = y.off;
                if (f16) gs.b_amax = g->amax + cs.qamax_slot[stp.y.id];
              } else {
                if (f16 && yslot) {
                  gs.b_amax = yslot;
                } else if (f16) {
                  gs.b_amax = g->amax + 1;
                  g->prof.begin("absmax", 0, 8.0 * N * K * nb, s);
                  dev::absmax(y.base, N * K * nb, g->amax + 1, next_amax_tag(g, s), s);
                  g->prof.end(s);
                }
                if (gather_y) {
                  gs.Bc = y.base;
                  gs.b_bs = y.bs;
                  gs.gb = cs.gy[k];
                } else {
                  g->prof.begin("split_permute", 0, 16.0 * N * K * nb, s);
                  dev::split_permute(y.base, sb, nb, cs.sy[k], stp.kb, gs.b_amax, s);
                  g->prof.end(s);
                  if (final) st.permute_bytes += 16.0 * N * K * nb, ++st.n_permute;
                  gs.B = sb;
                  gs.b_bs = N * K;
                }
              }
              const Node& out = P.nodes[stp.out];
              gs.C = arena + out.offset * B;
              gs.c_bs = out.elems();
              gs.M = M;
              gs.N = N;
              gs.K = K;
              gs.batch = nb;
              if (f16 && cs.node_slot[stp.out] >= 0) {
                gs.c_amax = g->node_amax + cs.node_slot[stp.out];
                gs.c_tag = next_amax_tag(g, s);
              }
              // algorithmic flops, 8 per complex multiply-add as for every product (the
              // kernel's own 16-bit MFMA work is a multiple of it that depends on its form)
              g->prof.begin(dev::gemm_split_name(gs), stp.flops() * nb,
                            8.0 * nb * (double)(M * K + N * K + M * N), s);
              dev::gemm_split(gs, s);
              g->prof.end(s);
              if (final) st.flops += stp.flops() * nb, ++st.n_gemm;
            };
            if (is_split) {
              int choice = cs.tuned[k];
              // a choice made before for this device, shape and operand sources
              const std::string tkey =
                  g->autotune ? g->device_sig + "|split" + (g->amax ? "16" : "bf") + "|" +
                                    std::to_string(M) + "x" + std::to_string(N) + "x" +
                                    std::to_string(K) + "|b" + std::to_string(nb) + "|g" +
                                    std::to_string((int)cs.gather_x[k]) +
                                    std::to_string((int)cs.gather_y[k]) + "|q" +
                                    std::to_string((int)stp.x.qubit) +
                                    std::to_string((int)stp.y.qubit) + "|c" +
                                    std::to_string(cs.xcache_offset[k] >= 0 ? 1 : 0)
                              : std::string();
              if (choice < 0 && g->autotune && tune_cache_get(tkey, &choice))
                cs.tuned[k] = choice;
              if (choice < 0 && g->autotune) {
                // time every fitting (tile, gathered x, gathered y) once on this call's operands
                dev::GemmSplit shape;
                shape.M = M;
                shape.N = N;
                shape.K = K;
                float best = 0;
                for (int gy = 0; gy < (cs.gather_y[k] ? 2 : 1); ++gy)
                  for (int gth = 0; gth < (cs.gather_x[k] ? 2 : 1); ++gth)
                    for (int t = 0; t < dev::kSplitTiles; ++t) {
                      if (!dev::gemm_split_tile_fits(shape, t)) continue;
                      const float ms =
                          time_launches([&] { run_split(gth == 1, gy == 1, t, false); });
                      if (choice < 0 || ms < best) choice = 4 * t + 2 * gy + gth, best = ms;
                    }
                cs.tuned[k] = choice;
                if (choice >= 0) tune_cache_put(tkey, choice);
              }
              if (choice >= 0) {
                run_split(choice & 1, (choice >> 1) & 1, choice >> 2, true);
              } else {
                // shape rules: a gathered operand is read again for every output tile along
                // the other dimension and split while staging; from 8192 rows (columns) on,
                // splitting it once and reading the compact layout costs less (32768^3: the
                // 3-multiplication 256x128 tile 515-518 against 545-547 ms per launch gathered,
                // the split pass of 2^30 elements about 3 ms; at 4096 the two are about even)
                run_split(cs.gather_x[k] != 0 && N < 8192, cs.gather_y[k] != 0 && M < 8192, -1,
                          true);
              }
              continue;
            }
            const bool gather_x = !cs.gather_x.empty() && cs.gather_x[k];
            if (stp.scratch_x >= 0 && !gather_x) {
              if (stp.x.qubit) fail(QFLEX_E_DEVICE, "internal: permutation of a qubit tensor");
              float2* dst = arena + P.nodes[stp.scratch_x].offset * B;
              g->prof.begin("permute", 0, 16.0 * (double)P.nodes[stp.scratch_x].elems() * nb, s);
              dev::permute(x.base, dst, nb, cs.px[k], s);
              g->prof.end(s);
              x.base = dst;
              st.permute_bytes += 16.0 * (double)P.nodes[stp.scratch_x].elems() * nb;
              ++st.n_permute;
            }
            if (stp.scratch_y >= 0) {
              if (stp.y.qubit) fail(QFLEX_E_DEVICE, "internal: permutation of a qubit tensor");
              float2* dst = arena + P.nodes[stp.scratch_y].offset * B;
              g->prof.begin("permute", 0, 16.0 * (double)P.nodes[stp.scratch_y].elems() * nb, s);
              dev::permute(y.base, dst, nb, cs.py[k], s);
              g->prof.end(s);
              y.base = dst;
              st.permute_bytes += 16.0 * (double)P.nodes[stp.scratch_y].elems() * nb;
              ++st.n_permute;
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
            const Node& out = P.nodes[stp.out];
            gm.C = arena + out.offset * B;
            gm.c_bs = out.elems();
            gm.M = M;
            gm.K = K;
            gm.N = N;
            gm.ta = stp.ta;
            gm.tb = stp.tb;
            gm.lda = stp.ta ? gm.M : gm.K;
            gm.ldb = stp.tb ? gm.K : gm.N;
            gm.ldc = gm.N;
            gm.batch = nb;
            if (gather_x) {  // x in its own storage order, on the MFMA rows kernel
              gm.gather = true;
              gm.ga = cs.gx[k];
              gm.ta = 0;
              gm.lda = gm.K;
              gm.force_variant = 8;
            } else {
              gm.force_variant = cs.tuned[k];
              if (gm.force_variant < 0 && g->autotune)  // time every fitting kernel variant once
                gm.force_variant = cs.tuned[k] = tune_gemm(g, s, gm);
            }
            g->prof.begin(dev::gemm_name(gm), stp.flops() * nb,
                          8.0 * nb * (double)(gm.M * gm.K + gm.K * gm.N + gm.M * gm.N), s);
            dev::gemm(gm, s);
            g->prof.end(s);
            st.flops += stp.flops() * nb;
            ++st.n_gemm;
          }
          View r = view(P.result);
          g->prof.begin("accumulate", 0, 40.0 * namp * nb, s);
          dev::accumulate(r.base, r.off, r.bs, r.add, namp, g->bidx + cs.bidx_offset,
                          acc + b0 * namp, namp, nb, s);
          g->prof.end(s);
        }
        // what the arena holds once this batch is done
        rs.valid = !slices.empty() && !graph;
        rs.circuit = c;
        rs.batch = B;
        rs.bits.assign(batch_bits, batch_bits + batch_bytes);
        rs.digits = digit;
        rs.arena = g->arena.p;
        rs.cache = g->split_cache.p;
      }
      st.n_slices += (int64_t)slices.size();
      st.n_bitstrings += nbs;
    }
  };
  try {
    if (!replayed) enqueue();
    if (capturing) {
      g->graph_stats = st;
      end_capture(true);
    }
  } catch (...) {
    rs.valid = false;
    if (capturing) end_capture(false);
    throw;
  }
  if (graph && s != s_user) {  // the caller's later work waits for the graph
    QHIP(hipEventRecord(g->graph_out, s));
    QHIP(hipStreamWaitEvent(s_user, g->graph_out, 0));
    s = s_user;
  }
  if (amp_total > 0 && !direct) {
    QHIP(hipMemcpyAsync(amps, acc_all, sizeof(double2) * amp_total,
                        amps_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!amps_on_device) QHIP(hipStreamSynchronize(s));
  }
  if (g->prof.on) {
    QHIP(hipStreamSynchronize(s));
    g->prof.resolve();
  }
  st.n_tuned = g->n_tuned - tuned0;
  g->last = st;
}

}  // namespace qflex
