// The program of the fused small-plan contraction (dev::fused_contract), built on the host
// from a contraction plan alone: qubit and step descriptors and the steps' index tables.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"

namespace qflex {

struct FusedProgram {
  std::vector<dev::FusedStep> steps;
  std::vector<dev::FusedQubit> qubits;  // grid_off left 0: the caller places the tensors
  std::vector<uint16_t> tables;
  dev::FusedPlan header;  // sizes and offsets; the device pointers are the caller's
  int64_t lds_bytes = 0;  // dynamic LDS per workgroup: image, step descriptors, tables
};

// Builds the program of plan P, or returns why it does not fit the kernel (empty when it
// fits).  LDS holds the plan's arena (intermediates at their arena offsets), then the free
// part of every qubit tensor, then the step descriptors and index tables; each step reads
// its operands through the storage positions of their labels.  Every offset and index is
// checked here against the LDS and tensor sizes.
std::string build_fused_program(const Plan& P, const Model& m, FusedProgram& prog);

// JSON object describing the fit: {"fits":1,"lds_bytes":..,"steps":..,"table_entries":..}
// or {"fits":0,"why":".."}.
std::string describe_fused(const Plan& P, const Model& m);

}  // namespace qflex
