// Circuit validation and the per-qubit time lines (paper, Methods A and B).
#include "model.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <set>

namespace qflex {

std::vector<cdouble> gate_matrix(int kind, double theta, double phi, const double* mat) {
  const double s2 = 1.0 / std::sqrt(2.0);
  const cdouble I(0, 1);
  switch (kind) {
    case QFLEX_G_H: return {s2, s2, s2, -s2};
    case QFLEX_G_X12: return {0.5 * (1.0 + I), 0.5 * (1.0 - I), 0.5 * (1.0 - I), 0.5 * (1.0 + I)};
    case QFLEX_G_Y12: return {0.5 * (1.0 + I), -0.5 * (1.0 + I), 0.5 * (1.0 + I), 0.5 * (1.0 + I)};
    case QFLEX_G_T: return {1.0, 0.0, 0.0, std::exp(I * (M_PI / 4))};
    case QFLEX_G_CZ: {
      std::vector<cdouble> m(16, 0.0);
      m[0] = m[5] = m[10] = 1.0;
      m[15] = -1.0;
      return m;
    }
    case QFLEX_G_FSIM: {
      std::vector<cdouble> m(16, 0.0);
      const double c = std::cos(theta), s = std::sin(theta);
      m[0] = 1.0;
      m[5] = c;
      m[6] = -I * s;
      m[9] = -I * s;
      m[10] = c;
      m[15] = std::exp(-I * phi);
      return m;
    }
    case QFLEX_G_MAT1:
    case QFLEX_G_MAT2: {
      const int d = kind == QFLEX_G_MAT1 ? 4 : 16;
      std::vector<cdouble> m(d);
      for (int i = 0; i < d; ++i) m[i] = cdouble(mat[2 * i], mat[2 * i + 1]);
      return m;
    }
  }
  fail(QFLEX_E_INVALID, "unknown gate kind " + std::to_string(kind));
}

static bool two_qubit(int kind) {
  return kind == QFLEX_G_CZ || kind == QFLEX_G_FSIM || kind == QFLEX_G_MAT2;
}

Model build_model(const qflex_circuit& c) {
  Model M;
  if (c.n_qubits < 1 || c.n_qubits > 4096) fail(QFLEX_E_INVALID, "n_qubits must be in [1, 4096]");
  if (!c.xy) fail(QFLEX_E_INVALID, "xy is NULL");
  if (c.n_gates < 0 || (c.n_gates > 0 && !c.gates)) fail(QFLEX_E_INVALID, "gates is NULL");
  M.n = c.n_qubits;
  std::set<std::pair<int, int>> seen;
  std::map<std::pair<int, int>, int> at;
  for (int q = 0; q < M.n; ++q) {
    std::pair<int, int> p(c.xy[2 * q], c.xy[2 * q + 1]);
    if (!seen.insert(p).second) fail(QFLEX_E_INVALID, "qubit coordinates repeated");
    M.xy.push_back(p);
  }
  // validate gates
  std::map<std::pair<int, int>, int> used;  // (cycle, qubit) -> gate index
  for (int64_t i = 0; i < c.n_gates; ++i) {
    const qflex_gate& g = c.gates[i];
    const std::string who = "gate " + std::to_string(i) + ": ";
    if (g.kind < QFLEX_G_H || g.kind > QFLEX_G_MAT2) fail(QFLEX_E_INVALID, who + "unknown kind");
    if (g.cycle < 0) fail(QFLEX_E_INVALID, who + "negative cycle");
    if (g.q0 < 0 || g.q0 >= M.n) fail(QFLEX_E_INVALID, who + "qubit id out of range");
    if ((g.kind == QFLEX_G_MAT1 || g.kind == QFLEX_G_MAT2) && !g.mat)
      fail(QFLEX_E_INVALID, who + "matrix is NULL");
    if (two_qubit(g.kind)) {
      if (g.q1 < 0 || g.q1 >= M.n || g.q1 == g.q0)
        fail(QFLEX_E_INVALID, who + "bad second qubit");
      const auto a = M.xy[g.q0], b = M.xy[g.q1];
      if (std::abs(a.first - b.first) + std::abs(a.second - b.second) != 1)
        fail(QFLEX_E_INVALID, who + "qubits are not at unit distance");
    } else if (g.q1 != -1) {
      fail(QFLEX_E_INVALID, who + "one-qubit gate with q1 != -1");
    }
    for (int q : {g.q0, g.q1}) {
      if (q < 0) continue;
      if (!used.emplace(std::make_pair(g.cycle, q), (int)i).second)
        fail(QFLEX_E_INVALID, who + "qubit " + std::to_string(q) + " used twice in cycle " +
                                  std::to_string(g.cycle));
    }
    for (double v : {g.theta, g.phi})
      if (!std::isfinite(v)) fail(QFLEX_E_INVALID, who + "non-finite angle");
    if (g.mat) {
      const int d = g.kind == QFLEX_G_MAT1 ? 8 : (g.kind == QFLEX_G_MAT2 ? 32 : 0);
      for (int j = 0; j < d; ++j)
        if (!std::isfinite(g.mat[j])) fail(QFLEX_E_INVALID, who + "non-finite matrix entry");
    }
    Gate G;
    G.cycle = g.cycle;
    G.kind = g.kind;
    G.q0 = g.q0;
    G.q1 = two_qubit(g.kind) ? g.q1 : -1;
    G.theta = g.theta;
    G.phi = g.phi;
    G.m = gate_matrix(g.kind, g.theta, g.phi, g.mat);
    M.gates.push_back(std::move(G));
  }
  // time order (stable: gates of one cycle act on disjoint qubits, so their order is moot)
  std::vector<int> order(M.gates.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return M.gates[a].cycle < M.gates[b].cycle; });
  M.timeline.assign(M.n, {});
  for (int gi : order) {
    const Gate& g = M.gates[gi];
    if (g.q1 < 0) {
      Piece p;
      p.gate = gi;
      p.mat = (int)(M.mats.size() / 4);
      for (int j = 0; j < 4; ++j) M.mats.push_back(g.m[j]);
      M.timeline[g.q0].push_back(p);
      continue;
    }
    // matrix in the |lo hi> basis
    const int lo = std::min(g.q0, g.q1), hi = std::max(g.q0, g.q1);
    std::vector<cdouble> m = g.m;
    if (g.q0 > g.q1) {
      static const int sw[4] = {0, 2, 1, 3};
      for (int r = 0; r < 4; ++r)
        for (int s = 0; s < 4; ++s) m[r * 4 + s] = g.m[sw[r] * 4 + sw[s]];
    }
    auto blk = [&](int i, int j, int a, int b) { return m[(2 * i + a) * 4 + (2 * j + b)]; };
    bool off_zero = true;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        off_zero = off_zero && blk(0, 1, a, b) == 0.0 && blk(1, 0, a, b) == 0.0;
    auto key = std::make_pair(lo, hi);
    auto it = M.link_of.find(key);
    int li;
    if (it == M.link_of.end()) {
      li = (int)M.links.size();
      M.link_of[key] = li;
      Link L;
      L.lo = lo;
      L.hi = hi;
      M.links.push_back(L);
    } else {
      li = it->second;
    }
    Link& L = M.links[li];
    const int rank = off_zero ? 2 : 4;
    Piece pl, ph;
    pl.gate = ph.gate = gi;
    pl.link = ph.link = li;
    pl.kbits = ph.kbits = off_zero ? 1 : 2;
    pl.koff = ph.koff = L.bits;
    ph.hi_side = true;
    L.gate_ids.push_back(gi);
    L.rank.push_back(rank);
    L.bits += pl.kbits;
    pl.mat = (int)(M.mats.size() / 4);
    for (int k = 0; k < rank; ++k) {  // A_k on the low qubit
      const int i = off_zero ? k : k >> 1, j = off_zero ? k : k & 1;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) M.mats.push_back((a == i && b == j) ? 1.0 : 0.0);
    }
    ph.mat = (int)(M.mats.size() / 4);
    for (int k = 0; k < rank; ++k) {  // B_k = G_ij on the high qubit
      const int i = off_zero ? k : k >> 1, j = off_zero ? k : k & 1;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) M.mats.push_back(blk(i, j, a, b));
    }
    M.timeline[lo].push_back(pl);
    M.timeline[hi].push_back(ph);
  }
  M.qlinks.assign(M.n, {});
  for (int li = 0; li < (int)M.links.size(); ++li) {
    M.qlinks[M.links[li].lo].push_back(li);
    M.qlinks[M.links[li].hi].push_back(li);
  }
  for (int q = 0; q < M.n; ++q)
    std::sort(M.qlinks[q].begin(), M.qlinks[q].end(),
              [&](int a, int b) { return M.other(a, q) < M.other(b, q); });
  return M;
}

}  // namespace qflex
