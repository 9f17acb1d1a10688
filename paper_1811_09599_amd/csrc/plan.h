// Contraction plan: which bonds are cut, in which order tensors are contracted pairwise, how
// each operand is laid out (and permuted when it must be), and where every intermediate
// lives in the device arena.
//
// Every tensor index here is binary: a link bond of 2^b values is b binary labels (most
// significant first) and a qubit's open output bit is one label.  A tensor layout is the
// list of its labels in storage order, most significant first (row-major).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "model.h"

namespace qflex {

struct QubitLayout {
  std::vector<int> storage;   // labels in storage order: fixed labels first, then free ones
  int n_fixed = 0;            // leading fixed labels (closed output bit, cut bonds)
  int out_shift = -1;         // bit position (from the LSB) of the output label; -1 if open
  std::vector<std::pair<int, int>> cut_shift;  // (cut index, bit position of its LSB)
  uint32_t deps = 0;          // cuts this tensor depends on
  int free_bits() const { return (int)storage.size() - n_fixed; }
};

struct Operand {
  bool qubit = false;  // qubit tensor view, else an intermediate node
  int id = -1;
};

struct PermDesc {
  int nbits = 0;
  std::vector<int> perm;  // perm[j] = input bit position feeding output bit position j (LSB=0)
};

struct Step {
  Operand x, y;
  int out = -1;                 // node produced
  int scratch_x = -1, scratch_y = -1;  // scratch node receiving a permuted operand, or -1
  PermDesc px, py;
  bool ta = false, tb = false;  // operand stored transposed ([K][M] / [N][K])
  int mb = 0, kb = 0, nb = 0;   // log2 of M, K, N
  uint32_t deps = 0;
  // label orders of the product: rows (M), contracted (K), columns (N); and the storage
  // orders of x and y as they come in (free labels only for qubit tensors)
  std::vector<int> mlab, klab, nlab, x_in, y_in;
  double flops() const { return 8.0 * std::ldexp(1.0, mb + kb + nb); }
};

struct Node {
  std::vector<int> labels;
  uint32_t deps = 0;
  int producer = -1, last_use = -1;
  bool persistent = false;
  int64_t offset = 0;  // elements, per bit-string, inside the arena
  int64_t elems() const { return int64_t(1) << labels.size(); }
};

struct Plan {
  int kind = QFLEX_PLAN_SWEEP;
  std::vector<int> cuts;       // link ids, slice-radix order (first most significant)
  std::vector<int> cut_bits;
  int total_link_bits = 0;     // labels [0, total_link_bits) are link bits
  std::vector<int> link_base;  // first label of each link
  std::vector<QubitLayout> qubits;
  std::vector<Node> nodes;
  std::vector<Step> steps;
  Operand result;              // tensor holding the open-qubit batch at the end
  std::vector<int> result_labels;
  std::vector<int> open;       // open qubit ids in the caller's order
  std::vector<uint32_t> batch_index;  // result element -> open-batch index (big-endian)
  int max_bits = 0;
  int64_t arena_elems = 0;     // per bit-string
  double flops_all_slices = 0; // per bit-string, f = 1, with reuse across slices
  // estimated seconds per bit-string at f = 1 (the automatic plan choice compares these):
  // every step, as often as it runs over the slices, at the slower of its arithmetic (at
  // the sustained rate of the kernel class its shape gets) and its memory traffic (operands,
  // result and permuted copies at the device's streaming rate)
  double cost_estimate = 0;

  int out_label(int q) const { return total_link_bits + q; }
  int64_t num_slices() const {
    int b = 0;
    for (int c : cut_bits) b += c;
    return int64_t(1) << b;
  }
  std::string describe(const Model& m) const;
};

Plan make_plan(const Model& m, const qflex_options& opt);

// Memory of the adjoint contraction of one slice, per bit-string, in complex elements.  The
// steps are cut into segments of consecutive steps.  The forward pass keeps only the
// intermediates that a later segment consumes (the checkpoints) and the whole last segment;
// the reverse sweep takes the segments last to first, recomputes each one (but the last) from
// the checkpoints and the qubit tensors, and reverses its steps.  Every step is recomputed at
// most once; the segmentation is the one with the least memory (checkpoint values and
// cotangents, plus the largest segment's values and cotangents, plus the cotangent scratch of
// one product's two operands), fewer segments on ties.
struct GradLayout {
  std::vector<std::pair<int, int>> segs;  // [first, end) steps of each segment, in order
  std::vector<char> ckpt;                 // per node: a checkpoint
  std::vector<int64_t> voff, coff;        // per node: value / cotangent offset, -1 if none
  int64_t s1off = 0, s2off = 0;           // cotangent scratch of a product's x and of its y
  int64_t elems = 0;                      // everything, per bit-string
  int64_t ckpt_elems = 0;                 // checkpoint values and cotangents
  int64_t segment_elems = 0;              // the largest segment's values and cotangents
  int64_t store_all_elems = 0;            // keeping every value and cotangent instead
  double recompute_flops = 0;             // products run again (segments but the last)
};
GradLayout make_grad_layout(const Plan& P, int64_t namp);

// Permutation taking a tensor stored with labels `in` to storage order `out` (same labels).
PermDesc make_perm_desc(const std::vector<int>& in, const std::vector<int>& out);

}  // namespace qflex
