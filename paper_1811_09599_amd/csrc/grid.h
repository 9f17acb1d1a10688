// The qflex_grid handle: per-circuit models, plans and device-resident qubit tensors, plus
// the device arena and staging buffers reused by contract calls.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "kernels.h"
#include "model.h"
#include "plan.h"

namespace qflex {

struct CircuitState {
  Model model;
  Plan plan;
  int64_t qdesc_base = 0;            // first GridQubit of this circuit in the device table
  int max_nlb = 0;
  int mat_base = 0;                  // first 2x2 matrix of this circuit in the device table
  int64_t grid_offset = 0;           // element offset of this circuit's qubit tensors
  std::vector<int64_t> qubit_offset; // element offset of each qubit tensor (within the grid)
  int64_t bidx_offset = 0;           // offset of its batch-index table in the device table
  std::vector<dev::PermTile> px, py; // per step (valid when the step permutes x / y)
  // split-precision products
  std::vector<char> split;           // per step: runs as a split (16-bit) product
  std::vector<dev::PermTile> sx, sy; // per step: node operand -> split operand layout
  std::vector<char> gather_x;        // per step: x read from complex64 storage by the product
  std::vector<dev::SplitGather> gx;  // per step: its gather descriptor
  std::vector<char> gather_y;        // per step: y read from complex64 storage by the product
  std::vector<dev::SplitGather> gy;  // per step: its gather descriptor
  // per step: x is an intermediate reused across slices, kept split in split_cache (offset in
  // 16-bit values per bit-string, -1 if not) and re-split only when it is recomputed
  std::vector<int64_t> xcache_offset;
  std::vector<int64_t> xcache_slot;  // its fp16 scale slot
  // fp16: per node, its slot in node_amax when a split product produces it (the product
  // records its largest magnitude, so consumers need no absmax pass), else -1
  std::vector<int64_t> node_slot;
  int64_t xcache_elems = 0;          // 16-bit values per bit-string
  // per step: the autotuner's choice (-1 untuned): split steps 2*tile + gather, complex64
  // steps the kernel variant; and for the adjoint, per step its forward, Xbar and Ybar products
  std::vector<int> tuned;
  std::vector<int> tuned_grad;
  // the fused small-plan program (device tables in qflex_grid::fused_prog), when the plan fits
  dev::FusedPlan fused;
  bool fused_ok = false;
  std::vector<int64_t> qsplit_offset;// per qubit: offset in grid_split (16-bit values), -1 if none
  std::vector<int64_t> qamax_slot;   // per qubit: fp16 scale slot in amax, -1 if none
  int64_t split_a_elems = 0, split_b_elems = 0;  // scratch per bit-string (16-bit values)
  GradLayout grad_layout;            // the adjoint's memory layout (made on first use)
  bool grad_layout_ready = false;
};

// Device buffer that only grows; freed with the grid.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void reserve(size_t n);  // throws Error(QFLEX_E_NOMEM / QFLEX_E_DEVICE)
  void release();
};

// Launch timing (qflex_set_profiling): events bracket each launch; durations are summed per
// kernel name once the call's work has finished.
struct Profiler {
  struct Rec {
    const char* name;
    hipEvent_t a, b;
    double flops, bytes;
  };
  struct Sum {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> pending;
  std::map<std::string, Sum> sums;
  hipEvent_t take();
  void begin(const char* name, double flops, double bytes, hipStream_t s);
  void end(hipStream_t s);
  void resolve();  // after the stream has finished
  void release();
};

// Pre-split of one qubit tensor for 16-bit products (made at grid build, repeated when the
// circuit's gates are updated).
struct QubitSplitJob {
  int circuit = 0;
  int64_t src = 0, dst = 0;  // grid element offset, grid_split offset (16-bit values)
  int nfixed = 0, nbits = 0, kbits = 0;
  dev::PermTile tile;
  int64_t slot = -1;         // fp16 scale slot, -1 for bf16
};

struct HostPinned {
  void* p = nullptr;
  size_t bytes = 0;
  void reserve(size_t n);
  void release();
};

// What the arena holds after a contract call: the circuit and bit-strings of the last batch
// contracted, the cut values of its last slice and the buffers it used.  Intermediates reused
// across slices live in a part of the arena of their own, so a later call whose first batch
// has the same circuit and bit-strings (and the same buffers) keeps every intermediate that
// depends on no cut whose value has changed, as a later slice of the same call would.
struct Resume {
  bool valid = false;
  int circuit = -1;
  int64_t batch = 0;              // bit-strings per batch the arena was laid out for
  std::vector<uint8_t> bits;      // the batch's bit-string rows
  std::vector<int64_t> digits;    // cut values of the last slice
  const void* arena = nullptr;
  const void* cache = nullptr;
};

}  // namespace qflex

struct qflex_grid {
  int device = 0;
  std::string device_sig;                // architecture and compute units (autotuner keys)
  int precision = QFLEX_PREC_C64;
  int bitstring_batch = 0;
  int slice_mode = QFLEX_SLICES_RANDOM;
  // graph mode: the captured launches of the last call and the call shape they belong to
  bool graph_mode = false;
  bool autotune = false;                 // time kernel variants per step on first use
  int fused_opt = 0;                     // qflex_options.fused: 0 where the plan fits, 1 required, -1 never
  int64_t n_tuned = 0;                   // kernel variants timed so far (time_launches calls)
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t graph_stream = nullptr;    // captures and replays (the null stream cannot capture)
  hipEvent_t graph_in = nullptr, graph_out = nullptr;
  std::string graph_key;
  qflex_stats graph_stats{};
  // the same for qflex_contract_grad (calls with one slice per circuit)
  hipGraphExec_t grad_graph_exec = nullptr;
  std::string grad_graph_key;
  qflex_stats grad_graph_stats{};
  bool grad_tuned = false;               // an autotuning gradient call has run
  std::vector<qflex::CircuitState> circ;
  float2* grid = nullptr;                // all qubit tensors
  int64_t grid_elems = 0;
  uint32_t* bidx = nullptr;              // batch-index tables of all circuits
  uint16_t* grid_split = nullptr;        // qubit tensors pre-split for 16-bit products
  // fp16 split scales: absmax slots [0] = row operand, [1] = column operand of the current
  // step, then one per pre-split qubit tensor; amax_tag = the last tag used on them
  uint64_t* amax = nullptr;
  int64_t n_amax = 0;
  uint64_t* node_amax = nullptr;         // node slots (see CircuitState::node_slot)
  int64_t n_node_amax = 0;
  uint32_t amax_tag = 0;
  // time-collapse descriptors, kept for the adjoint of the grid build
  qflex::DevBuf gq, gpieces, gmats, gpos;
  std::vector<qflex::QubitSplitJob> qsplit_jobs;
  int64_t n_mats = 0;
  int max_pieces = 0;                    // longest qubit time line
  // gradient buffers
  qflex::DevBuf grad_arena, tbar, pbar, gbar, amps_dev, xeb;
  qflex::DevBuf splitk_ws;               // partial products of split-K complex64 products
  qflex::DevBuf fs_buf;                  // qflex_fidelity_samples: amplitudes, draws, results
  qflex::DevBuf split_scratch;           // split operands of intermediates
  qflex::DevBuf split_cache;             // split copies of intermediates reused across slices
  qflex::DevBuf arena;                   // intermediates
  qflex::DevBuf amps64;                  // FP64 amplitude accumulator
  qflex::DevBuf offs;                    // per-bit-string output offsets of the qubit tensors
  qflex::DevBuf fused_prog;              // fused small-plan programs: steps, then qubit tables
  qflex::HostPinned offs_host;
  qflex::HostPinned grad_host;           // piece cotangents and cross-entropy sums, on the host
  hipEvent_t offs_done = nullptr;        // the last upload out of offs_host has finished
  // offsets tables that fused kernels read in place from host memory (no upload), used in
  // turn; each one's event is recorded after the launches of the call that read it
  qflex::HostPinned offs_pinned[2];
  void* offs_pinned_dev[2] = {nullptr, nullptr};   // their device addresses
  const void* offs_pinned_at[2] = {nullptr, nullptr};  // the host buffer those belong to
  hipEvent_t offs_pinned_done[2] = {nullptr, nullptr};
  int offs_pinned_next = 0;
  // the current call's offsets table (device address) and the pinned buffer it is, or -1
  const int64_t* offs_cur = nullptr;
  int offs_pinned_slot = -1;
  qflex_stats last{};
  qflex::Profiler prof;
  qflex::Resume resume;                  // intermediates kept from the last contract call
};

namespace qflex {
void build_grid_device(qflex_grid* g, hipStream_t s);
// New gates for circuit c (same qubits, couplers, cycles, kinds and bond ranks): its qubit
// tensors are collapsed again (and split again for 16-bit products); plan, tuned kernels and
// buffers stay.
void update_gates(qflex_grid* g, int c, const qflex_circuit& circuit, hipStream_t s);
// Host checks of a contract call, the slices each circuit sums, and the per-bit-string
// output offsets of the qubit tensors (g->offs_cur): uploaded to g->offs, or, when
// `pinned_ok` and every circuit of the call runs the fused kernel, written into one of the
// pinned buffers that the kernel reads in place (g->offs_pinned_slot; the caller records
// that buffer's event after its launches).  Everything contract() does before its launches.
std::vector<std::vector<int64_t>> prepare_call(qflex_grid* g, const uint8_t* bits,
                                               const int64_t* bs_offsets, double fidelity,
                                               uint64_t seed, const int64_t* slice_ids,
                                               const int64_t* slice_offsets, const void* amps,
                                               hipStream_t s, bool pinned_ok = false);
// Autotuning: the shortest of three timed runs of `launch` after a warm-up run (profiling off;
// the stream is synchronised), and the fastest kernel variant of a complex64 product.
float time_launches(qflex_grid* g, hipStream_t s, const std::function<void()>& launch);
int tune_gemm(qflex_grid* g, hipStream_t s, const dev::Gemm& gm);
// The process-wide table of autotuner choices (qflex_autotune_cache_*): keys name the device
// (device_signature) and everything the timing depended on.
std::string device_signature(int device);
bool tune_cache_get(const std::string& key, int* choice);
void tune_cache_put(const std::string& key, int choice);
void contract(qflex_grid* g, const uint8_t* bits, const int64_t* bs_offsets, double fidelity,
              uint64_t seed, const int64_t* slice_ids, const int64_t* slice_offsets,
              double* amps, int32_t out_flags, hipStream_t s);
std::vector<int64_t> select_slices(int64_t total, double fidelity, uint64_t seed, int mode);
void contract_grad(qflex_grid* g, const uint8_t* bits, const int64_t* bs_offsets,
                   double fidelity, uint64_t seed, const int64_t* slice_ids,
                   const int64_t* slice_offsets, const double* cot, int32_t cot_on_device,
                   double* amps, double* grad_gates, double* grad_params, double* loss,
                   bool out_on_device, hipStream_t s);
}  // namespace qflex
