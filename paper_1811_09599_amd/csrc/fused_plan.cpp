// Host builder of the fused small-plan contraction program (see fused_plan.h).
#include "fused_plan.h"

#include <algorithm>
#include <sstream>

namespace qflex {

std::string build_fused_program(const Plan& P, const Model& m, FusedProgram& prog) {
  std::vector<dev::FusedStep>& steps = prog.steps;
  std::vector<dev::FusedQubit>& qubits = prog.qubits;
  std::vector<uint16_t>& tables = prog.tables;
  if ((int)P.steps.size() > dev::kFusedMaxSteps) return "more than 128 steps";
  if (m.n > dev::kFusedMaxQubits) return "more than 128 qubits";
  if ((int)P.cuts.size() > dev::kFusedMaxCuts) return "more than 32 cuts";
  if (P.result.qubit) return "the result is a qubit tensor";
  int64_t lds = P.arena_elems;
  qubits.assign(m.n, dev::FusedQubit{});
  for (int q = 0; q < m.n; ++q) {
    const QubitLayout& L = P.qubits[q];
    dev::FusedQubit& fq = qubits[q];
    if ((int)L.cut_shift.size() > dev::kFusedMaxQubitCuts) return "a qubit tensor on > 8 cuts";
    if (L.free_bits() > dev::kFusedMaxBits) return "a qubit tensor too large";
    fq.free_bits = L.free_bits();
    fq.lds = (int32_t)lds;
    lds += int64_t(1) << L.free_bits();
    fq.out_row = L.out_shift >= 0 ? q : -1;
    fq.ncut = (int32_t)L.cut_shift.size();
    for (int j = 0; j < fq.ncut; ++j) {
      fq.cut[j] = (int8_t)L.cut_shift[j].first;
      fq.shift[j] = (int8_t)L.cut_shift[j].second;
    }
    fq.deps = L.deps;
    if (lds > dev::kFusedMaxLdsElems) return "more than 144 KiB of LDS per bit-string";
  }
  // operand: LDS offset, elements
  auto where = [&](const Operand& o) -> std::pair<int64_t, int64_t> {
    if (o.qubit) return {qubits[o.id].lds, int64_t(1) << qubits[o.id].free_bits};
    return {P.nodes[o.id].offset, P.nodes[o.id].elems()};
  };
  // storage bit positions of `logical` labels (least significant first) in `storage` (MSB
  // first); false if one is missing
  auto positions = [](const std::vector<int>& storage, const std::vector<int>& logical,
                      int8_t* pos) {
    const int n = (int)storage.size(), k = (int)logical.size();
    for (int j = 0; j < k; ++j) {
      const int label = logical[k - 1 - j];
      const auto it = std::find(storage.begin(), storage.end(), label);
      if (it == storage.end()) return false;
      pos[j] = (int8_t)(n - 1 - (int)(it - storage.begin()));
    }
    return true;
  };
  steps.assign(P.steps.size(), dev::FusedStep{});
  tables.clear();
  for (size_t k = 0; k < P.steps.size(); ++k) {
    const Step& st = P.steps[k];
    dev::FusedStep& fs = steps[k];
    int8_t xm[dev::kFusedMaxBits], xk[dev::kFusedMaxBits], yk[dev::kFusedMaxBits],
        yn[dev::kFusedMaxBits];
    if (st.kb > dev::kFusedMaxKBits) return "a step contracts more than 10 labels";
    if ((int)st.x_in.size() != st.mb + st.kb || (int)st.y_in.size() != st.kb + st.nb ||
        st.mb + st.kb > dev::kFusedMaxBits || st.kb + st.nb > dev::kFusedMaxBits)
      return "a step's operand labels do not match its product";
    std::vector<int> out_labels = st.mlab;
    out_labels.insert(out_labels.end(), st.nlab.begin(), st.nlab.end());
    if (P.nodes[st.out].labels != out_labels) return "a step's result is not stored [M][N]";
    if (!positions(st.x_in, st.mlab, xm) || !positions(st.x_in, st.klab, xk) ||
        !positions(st.y_in, st.klab, yk) || !positions(st.y_in, st.nlab, yn))
      return "a step's operand lacks one of its labels";
    const auto x = where(st.x), y = where(st.y);
    const int64_t out = P.nodes[st.out].offset, out_n = P.nodes[st.out].elems();
    if (x.second != (int64_t(1) << (st.mb + st.kb)) || y.second != (int64_t(1) << (st.kb + st.nb)))
      return "a step's operand size does not match its labels";
    auto overlap = [](int64_t a, int64_t an, int64_t b, int64_t bn) { return a < b + bn && b < a + an; };
    if (out < 0 || out + out_n > P.arena_elems || overlap(out, out_n, x.first, x.second) ||
        overlap(out, out_n, y.first, y.second))
      return "a step's result overlaps an operand";
    if (x.first < 0 || x.first + x.second > lds || y.first < 0 || y.first + y.second > lds)
      return "an operand outside the LDS image";
    fs.x = (int32_t)x.first;
    fs.y = (int32_t)y.first;
    fs.out = (int32_t)out;
    fs.mb = st.mb;
    fs.kb = st.kb;
    fs.nb = st.nb;
    fs.deps = st.deps;
    // index tables: an index is below its operand's size, which the 16-bit entries bound to
    // 2^16 elements (the LDS image itself holds fewer)
    if (x.second > 65536 || y.second > 65536) return "an operand of more than 2^16 elements";
    auto deposit = [](int64_t v, const int8_t* pos, int n) {
      int64_t o = 0;
      for (int j = 0; j < n; ++j) o |= ((v >> j) & 1) << pos[j];
      return (uint16_t)o;
    };
    const int64_t need = (int64_t(1) << st.mb) + (int64_t(1) << st.nb) + (int64_t(2) << st.kb);
    if ((int64_t)tables.size() + need > 4 * dev::kFusedMaxLdsElems) return "index tables too large";
    fs.tab = (int32_t)tables.size();
    for (int64_t i = 0; i < (int64_t(1) << st.mb); ++i) tables.push_back(deposit(i, xm, st.mb));
    for (int64_t i = 0; i < (int64_t(1) << st.nb); ++i) tables.push_back(deposit(i, yn, st.nb));
    for (int64_t i = 0; i < (int64_t(1) << st.kb); ++i) tables.push_back(deposit(i, xk, st.kb));
    for (int64_t i = 0; i < (int64_t(1) << st.kb); ++i) tables.push_back(deposit(i, yk, st.kb));
  }
  // the step descriptors and index tables follow the image in LDS (the kernel's launcher
  // sizes its dynamic LDS the same way)
  const int64_t bytes = (int64_t)sizeof(float2) * std::max<int64_t>(lds, 1) +
                        (int64_t)sizeof(dev::FusedStep) * (int64_t)steps.size() +
                        (int64_t)sizeof(uint16_t) * (int64_t)tables.size();
  if (bytes > (int64_t)sizeof(float2) * dev::kFusedMaxLdsElems)
    return "more than 144 KiB of LDS per bit-string with the step descriptors and tables";
  const int64_t namp = int64_t(1) << P.open.size();
  const auto r = where(P.result);
  if (r.first < 0 || r.first + namp > P.arena_elems || namp > r.second)
    return "the result tensor is outside the arena";
  dev::FusedPlan& fp = prog.header;
  fp = dev::FusedPlan{};
  fp.nsteps = (int32_t)steps.size();
  fp.nq = (int32_t)qubits.size();
  fp.ntab = (int32_t)tables.size();
  fp.lds_elems = (int32_t)std::max<int64_t>(lds, 1);
  fp.result = (int32_t)r.first;
  fp.namp = (int32_t)namp;
  fp.ncut = (int32_t)P.cuts.size();
  for (int c = 0; c < fp.ncut; ++c) fp.cut_bits[c] = (int8_t)P.cut_bits[c];
  prog.lds_bytes = bytes;
  return "";
}

std::string describe_fused(const Plan& P, const Model& m) {
  FusedProgram prog;
  const std::string why = build_fused_program(P, m, prog);
  std::ostringstream o;
  if (why.empty())
    o << "{\"fits\":1,\"lds_bytes\":" << prog.lds_bytes << ",\"steps\":" << prog.steps.size()
      << ",\"table_entries\":" << prog.tables.size() << "}";
  else
    o << "{\"fits\":0,\"why\":\"" << why << "\"}";  // the reasons hold no quote or backslash
  return o.str();
}

}  // namespace qflex
