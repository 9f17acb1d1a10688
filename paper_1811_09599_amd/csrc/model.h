// Host-side model of a circuit: validated gates, links (neighbouring qubit pairs that share
// gates), per-qubit time lines of 2x2 pieces, and the label space used by the planner.
#pragma once

#include <complex>
#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qflex.h"

namespace qflex {

using cdouble = std::complex<double>;

// Thrown by host code; api.cpp turns it into a status and a message.
struct Error : std::runtime_error {
  qflex_status status;
  Error(qflex_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(qflex_status s, const std::string& m) { throw Error(s, m); }

// One link = a pair of qubits (lo < hi) that share at least one two-qubit gate.  Its bond is
// the mixed-radix index over its gates' bond values, earliest gate most significant; every
// rank is 2 or 4, so the bond has `bits` binary digits.
struct Link {
  int lo = 0, hi = 0;
  std::vector<int> gate_ids;  // indices into Model::gates, time order
  std::vector<int> rank;      // 2 or 4 per gate
  int bits = 0;               // sum of log2(rank)
};

// A 2x2 piece of a qubit's time line: either a one-qubit gate (nk == 1) or the qubit's side
// of a two-qubit gate's bond decomposition (nk = rank, selected by the bond value k).
struct Piece {
  int gate = -1;   // index into Model::gates
  int link = -1;   // link id (bond pieces)
  int kbits = 0;   // log2(rank) (0 for one-qubit gates)
  int koff = 0;    // offset of this gate's k digits inside the link bond, from the MSB
  int mat = 0;     // index of the first 2x2 matrix in Model::mats
  bool hi_side = false;
};

struct Gate {
  int cycle = 0, kind = 0, q0 = -1, q1 = -1;
  double theta = 0, phi = 0;
  std::vector<cdouble> m;  // 2x2 or 4x4 row-major, basis ordered by (q0, q1) as given
};

struct Model {
  int n = 0;
  std::vector<std::pair<int, int>> xy;
  std::vector<Gate> gates;
  std::vector<Link> links;
  std::map<std::pair<int, int>, int> link_of;  // (lo, hi) -> link id
  std::vector<std::vector<int>> qlinks;        // per qubit: link ids by neighbour id
  std::vector<std::vector<Piece>> timeline;    // per qubit, time order
  std::vector<cdouble> mats;                   // 2x2 matrices, row-major, 4 entries each

  int other(int link, int q) const { return links[link].lo == q ? links[link].hi : links[link].lo; }
};

// Validate a circuit and build its model (throws Error(QFLEX_E_INVALID, ...)).
Model build_model(const qflex_circuit& c);

// Gate matrix of a validated gate description (basis ordered by (q0, q1)).
std::vector<cdouble> gate_matrix(int kind, double theta, double phi, const double* mat);

}  // namespace qflex
