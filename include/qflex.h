/*
 * qflex.h - C ABI of an MI355X (gfx950) library that computes amplitudes of random quantum
 * circuits (RQCs) on 2D qubit layouts by tensor-network contraction, after qFlex
 * (Villalonga et al., "A flexible high-performance simulator for verifying and
 * benchmarking quantum circuits implemented on real hardware", arXiv:1811.09599).
 *
 * What the calls compute (paper, Methods B and C.1):
 *   - A circuit with input |0...0> and output bit-string x is a tensor network whose value is
 *     the amplitude psi(x) = <x|U|0...0>.
 *   - qflex_build_grid collapses each qubit's gates along time into one tensor per qubit
 *     (Methods B.1: contraction in the time direction first, at negligible cost), leaving
 *     the output bit of every qubit open so that one grid serves every bit-string.
 *   - qflex_contract_amplitudes contracts the grid for given output bit-strings in a fixed
 *     pairwise order.  Each pairwise step is an index permutation followed by a complex
 *     matrix product (Methods B.2).  Cut bonds are fixed to explicit values ("paths") and
 *     the amplitude is the sum over paths (Methods B.1, cutting indexes); summing a
 *     fraction f of the paths yields fidelity-f amplitudes (Methods C.1, Eq. 1).  Qubits
 *     listed as open keep their output bit free, giving a batch of 2^n_open amplitudes per
 *     bit-string (Methods C.2 and SI A, fast sampling).
 *
 * Conventions
 *   - Qubit q's output bit in a bit-string row is bits[q] (0 or 1).
 *   - Two-qubit gate matrices are 4x4 in the basis |q0 q1> = 00, 01, 10, 11.
 *   - The bond of a two-qubit gate is its decomposition G = sum_k A_k (x) B_k in the
 *     elementary basis of the lower-id qubit: k in {0,1} (A_k = |k><k|) when both
 *     off-diagonal 2x2 blocks of G are exactly zero, else k = 2i+j (A_k = |i><j|).  A link's
 *     bond value is the mixed-radix index of its gates' k, earliest gate most significant.
 *   - A slice (path) id is the mixed-radix index of the cut links' bond values, in the
 *     order reported by qflex_plan_cuts (first cut most significant).
 *   - The open-qubit batch index is big-endian over open_qubits in the order given.
 *   - Amplitudes are complex128, interleaved (re, im).
 *
 * Ownership: the caller owns every input array; the library copies what it needs before a
 * call returns.  A qflex_grid owns all device memory it allocates until qflex_grid_free.
 * Output buffers are caller-allocated (device memory when *_on_device is 1, host memory
 * otherwise).
 *
 * Errors: every call validates its arguments before launching any GPU work.  On a non-OK
 * status, qflex_last_error() returns a message for the calling thread.  A grid handle may
 * not be used from two threads at once; distinct handles may.
 */
#ifndef QFLEX_H
#define QFLEX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QFLEX_OK = 0,
  QFLEX_E_INVALID = 1,     /* argument or circuit fails validation; nothing was launched */
  QFLEX_E_PLAN = 2,        /* no contraction plan fits max_tensor_elems, or fidelity*slices
                              is not an integer >= 1 */
  QFLEX_E_NOMEM = 3,       /* a device or host allocation failed */
  QFLEX_E_DEVICE = 4,      /* a HIP runtime error (also an asynchronous one from earlier work) */
  QFLEX_E_UNSUPPORTED = 5  /* valid request the library does not implement */
} qflex_status;

typedef enum {
  QFLEX_PREC_C64 = 0,        /* complex64 operands, FP32 MFMA, FP32 accumulation */
  QFLEX_PREC_SPLIT_BF16 = 1, /* complex64 operands split into hi+lo bf16, FP32 accumulation */
  QFLEX_PREC_SPLIT_FP16 = 2  /* hi+lo fp16 parts of the operand times a power-of-two scale */
} qflex_precision;

/* Gate kinds (matrices as in the paper's Methods A; fSim as in the comment below). */
typedef enum {
  QFLEX_G_H = 0,    /* (1/sqrt2)[[1,1],[1,-1]] */
  QFLEX_G_X12 = 1,  /* 1/2[[1+i,1-i],[1-i,1+i]] */
  QFLEX_G_Y12 = 2,  /* 1/2[[1+i,-1-i],[1+i,1+i]] */
  QFLEX_G_T = 3,    /* diag(1, e^{i pi/4}) */
  QFLEX_G_CZ = 4,   /* diag(1,1,1,-1) */
  QFLEX_G_FSIM = 5, /* [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,e^{-i phi}]] */
  QFLEX_G_MAT1 = 6, /* explicit 2x2 matrix in qflex_gate.mat */
  QFLEX_G_MAT2 = 7  /* explicit 4x4 matrix in qflex_gate.mat */
} qflex_gate_kind;

typedef enum {
  QFLEX_PLAN_AUTO = 0,     /* of SWEEP, QUADRANT (full rectangular grids) and CUT_SWEEP, the
                              kinds that fit max_tensor_elems, the one with the lowest
                              estimated time (qflex_plan_describe's cost_estimate_s: per step
                              and slice, the slowest of its flops at a sustained product rate,
                              its bytes at a streaming rate and its launches); ties go to the
                              earlier kind in that list */
  QFLEX_PLAN_SWEEP = 1,    /* absorb every qubit into one tensor, no cuts */
  QFLEX_PLAN_QUADRANT = 2, /* four regions A|B over C|D, one cut between B and D in the last
                              column and one between C and D in the last row (SI A) */
  QFLEX_PLAN_CUT_SWEEP = 3 /* any layout: one sweep in the qubit order with the narrowest
                              frontier, cutting links (most over-limit frontiers first) until
                              every intermediate fits max_tensor_elems (Methods B.1 cutting) */
} qflex_plan_kind;

typedef struct {
  int32_t cycle;     /* time step; gates of one cycle must act on disjoint qubits */
  int32_t kind;      /* qflex_gate_kind */
  int32_t q0, q1;    /* qubit ids; q1 = -1 for one-qubit gates */
  double theta, phi; /* fSim angles in radians (QFLEX_G_FSIM only) */
  const double* mat; /* MAT1: 2x2, MAT2: 4x4 complex128 interleaved row-major; else NULL */
} qflex_gate;

typedef struct {
  int32_t n_qubits;         /* 1 .. 4096 */
  const int32_t* xy;        /* [n_qubits][2] integer (row, col) coordinates, distinct; two
                               qubits may share a gate only if they are at unit distance */
  const qflex_gate* gates;  /* [n_gates] in any order */
  int64_t n_gates;
} qflex_circuit;

typedef struct {
  int32_t precision;         /* qflex_precision */
  int32_t plan_kind;         /* qflex_plan_kind */
  int64_t max_tensor_elems;  /* largest intermediate tensor per bit-string (0 = 2^30) */
  const int32_t* open_qubits;/* qubits whose output bit stays open (may be NULL) */
  int32_t n_open;            /* 0 .. 16; the same ids are used for every circuit */
  int32_t bitstring_batch;   /* most bit-strings contracted together (0 = automatic) */
  int32_t slice_mode;        /* subset summed at fidelity f < 1 (Methods C.1), k = f * S:
                                QFLEX_SLICES_RANDOM: k ids of a SplitMix64-driven Fisher-Yates
                                shuffle of [0, S), sorted;
                                QFLEX_SLICES_BLOCK: k must divide S; the k consecutive ids from
                                a seeded multiple of k (the leading cuts fixed, the trailing
                                ones all summed: intermediates reused across the block) */
  int32_t graph;             /* 1: qflex_contract_amplitudes captures its launches in one HIP
                                graph and replays it for later calls with the same shapes and
                                slices (bit-strings may differ), and so does
                                qflex_contract_grad for calls that sum one slice per circuit
                                (cotangents may differ too); capture and replay run on the
                                caller's stream, or on a stream of the grid's ordered after
                                the caller's when that is the null stream.  An autotuning grid
                                runs its first call eagerly.  A call whose circuits all run the
                                fused small-plan kernel is launched directly (one kernel per
                                circuit and 64 slices: a graph saves no launch).  0: launches
                                every call */
  int32_t autotune;          /* 1: the first call that runs a contraction step times every
                                kernel variant that fits it (product tiles, kernel family, and
                                for split products gathered vs permuted row operands) on that
                                call's operands and keeps the fastest for the grid's lifetime;
                                results do not depend on the choice beyond rounding order */
  int32_t fused;             /* complex64 grids: 0 (default) contracts every circuit whose plan
                                fits one workgroup's LDS per bit-string (intermediates and the
                                qubit tensors' free parts within 144 KiB, at most 128 steps,
                                at most 10 contracted labels per step, the result an
                                intermediate) in one kernel launch per call and up to 64 slices:
                                one workgroup per bit-string runs every step in LDS, its
                                operands read in place (no permutation), and adds the result
                                to the FP64 amplitudes; other circuits take the step-by-step
                                path.  1: every circuit must fit (QFLEX_E_INVALID at build
                                otherwise).  -1: never.  Split precisions ignore 0 and reject
                                1. */
} qflex_options;

typedef enum { QFLEX_SLICES_RANDOM = 0, QFLEX_SLICES_BLOCK = 1 } qflex_slice_mode;

/* Flags of qflex_contract_amplitudes' amps_on_device argument: 0 = host output, 1 = device
 * output, 1|2 = device output that the call adds its slice sums to instead of overwriting. */
typedef enum {
  QFLEX_OUT_HOST = 0,
  QFLEX_OUT_DEVICE = 1,
  QFLEX_OUT_ACCUMULATE = 2
} qflex_out_flags;

typedef struct qflex_grid qflex_grid;

/* Statistics of the most recent contract call on a grid (algorithmic counts). */
typedef struct {
  double flops;          /* 8 real flops per complex multiply-add of every matrix product run */
  double permute_bytes;  /* bytes read + written by index permutations */
  int64_t n_gemm;        /* matrix products launched */
  int64_t n_permute;     /* permutation kernels launched */
  int64_t n_slices;      /* slices summed, over all circuits */
  int64_t n_bitstrings;  /* bit-strings contracted, over all circuits */
  int64_t n_tuned;       /* kernel variants the autotuner timed during the call */
} qflex_stats;

/* Validate circuits (Methods A: gates of a cycle act on disjoint qubits, two-qubit gates on
 * nearest neighbours), plan their contractions (Methods B.1: cuts and pairwise order), collapse
 * every qubit's gates along time on the GPU (Methods B.1: the time direction is contracted
 * first; bond dimension = the Schmidt rank of each gate) and keep the per-qubit tensors in
 * device memory.  stream: a hipStream_t (NULL = the null stream).  Returns QFLEX_E_INVALID for: n_circuits < 1, a NULL pointer, coordinates
 * repeated, a qubit id out of range, a gate between qubits not at unit distance, a qubit used
 * twice in one cycle, an unknown kind, a missing matrix, n_open > 16 or an open id out of
 * range.  QFLEX_E_PLAN when no plan fits max_tensor_elems. */
qflex_status qflex_build_grid(const qflex_circuit* circuits, int32_t n_circuits,
                              const qflex_options* opt, void* stream, qflex_grid** out);

/* Replace the gates of circuit `circuit` of a grid by those of `updated` and collapse its qubit
 * tensors along time again (Methods B.1), e.g. for new fSim angles in a fitting loop.  The
 * update must keep the circuit's structure: the same qubits and coordinates, and gates of the
 * same kinds on the same qubits in the same cycles and order, with the same bond ranks (an fSim
 * gate whose off-diagonal blocks become exactly zero, theta = 0, changes rank).  The plan,
 * the autotuner's choices, graphs and buffers are kept; intermediates kept from earlier calls
 * are dropped.  stream: as for qflex_build_grid; the call returns when the tensors are
 * rebuilt.  QFLEX_E_INVALID (the grid unchanged) for a bad index, an invalid circuit or a
 * different structure. */
qflex_status qflex_update_gates(qflex_grid* g, int32_t circuit, const qflex_circuit* updated,
                                void* stream);

/* Number of slices S (paths) of circuit `circuit`'s plan (1 when it has no cuts). */
qflex_status qflex_num_slices(const qflex_grid* g, int32_t circuit, int64_t* total);

/* Cut links of circuit `circuit`'s plan, in slice-radix order (first = most significant):
 * pairs[2*i], pairs[2*i+1] = lower and higher qubit id of cut i.  At most max_cuts are
 * written; *n_cuts receives the count. */
qflex_status qflex_plan_cuts(const qflex_grid* g, int32_t circuit, int32_t* pairs,
                             int32_t max_cuts, int32_t* n_cuts);

/* Validate and plan one circuit without touching the GPU; writes a JSON description of the
 * plan (cuts, steps with their matrix-product shapes, label orders and flops per bit-string,
 * memory) into buf (NUL-terminated, truncated to len).  *needed receives the full length + 1.
 * A step's label lists (most significant first) are the product's rows, contracted labels and
 * columns (mlab, klab, nlab) and the storage orders of its operands as they come in (x_in,
 * y_in; free labels only for a qubit tensor).  "fused" tells whether the plan fits the fused
 * small-plan kernel (one workgroup per bit-string, every step in LDS; complex64 grids use it
 * unless qflex_options.fused is -1): {"fits":1,"lds_bytes","steps","table_entries"} or
 * {"fits":0,"why"}. */
qflex_status qflex_plan_describe(const qflex_circuit* circuit, const qflex_options* opt,
                                 char* buf, int64_t len, int64_t* needed);

/* Contract amplitudes: psi(x) summed over the selected paths (Methods B.1, cutting indexes:
 * the amplitude is the sum of the contributions of every value of the cut bonds; Methods C.1:
 * a fraction f of those paths gives a fidelity-f amplitude, Eq. 1; Methods C.2 and SI A: open
 * qubits give a batch of amplitudes per contraction).
 *   bits        uint8 rows, concatenated per circuit: circuit c contributes
 *               bs_offsets[c+1]-bs_offsets[c] rows of n_qubits(c) bytes each (host memory).
 *   bs_offsets  [n_circuits+1] prefix offsets of bit-string rows (host memory).
 *   fidelity    f in (0, 1]: k = f*S_c slices are summed for circuit c, chosen by SplitMix64
 *               (seed slice_seed) driving a Fisher-Yates shuffle of [0, S_c): for i from
 *               S_c-1 down to 1, j = next() mod (i+1), swap; the first k entries are used.
 *               Ignored when slice_ids is given.
 *   slice_ids, slice_offsets  optional explicit slice lists per circuit (host memory,
 *               concatenated; slice_offsets has n_circuits+1 entries), else NULL.
 *   amps        complex128 [total bit-strings][2^n_open] (device if amps_on_device).
 *   amps_on_device  qflex_out_flags: QFLEX_OUT_HOST, QFLEX_OUT_DEVICE, or
 *               QFLEX_OUT_DEVICE | QFLEX_OUT_ACCUMULATE to add this call's sums to amps
 *               (device) instead of overwriting them; any other value is QFLEX_E_INVALID.
 * The sum over slices is accumulated in FP64.
 * Reuse across calls: intermediates that depend on no cut, or only on cuts whose value is the
 * same, are computed once per bit-string batch and reused by the later slices of a call (SI A).
 * They stay in the grid's device memory after the call: when the next call's first batch
 * contracts the same circuit with the same bit-strings (same batch size), its first slice
 * reuses them as a later slice of the previous call would.  So the slices of one amplitude
 * batch may be spread over several accumulating calls at the cost of one call over all of
 * them (in ascending slice order; with QFLEX_SLICES_BLOCK subsets the per-right-cut
 * intermediates are then computed once).  Results do not depend on it.  Graph mode keeps
 * nothing across calls. */
qflex_status qflex_contract_amplitudes(qflex_grid* g, const uint8_t* bits,
                                       const int64_t* bs_offsets, double fidelity,
                                       uint64_t slice_seed, const int64_t* slice_ids,
                                       const int64_t* slice_offsets, double* amps,
                                       int32_t amps_on_device, void* stream);

/* Gradients of a real loss L of the amplitudes (adjoint contraction).
 *   bits ... slice_offsets   as for qflex_contract_amplitudes (the same slices are summed).
 *   cotangent  complex128 [total bit-strings][2^n_open] dL/dRe(amp) + i dL/dIm(amp) (the
 *              convention of PyTorch's complex autograd, = 2 dL/d(conj amp)), on the device if
 *              cotangent_on_device; or NULL for the linear cross-entropy of each circuit,
 *              F = (2^n/m) sum |amp|^2 - 1 over its m amplitudes, as the loss (summed over
 *              circuits).
 *   amps       complex128 [total bit-strings][2^n_open] amplitudes (may be NULL).
 *   grad_gates complex128 dL/dRe(G) + i dL/dIm(G) (same convention) for every entry of every
 *              gate, circuits in order and
 *              gates in their input order, 4 entries for a one-qubit gate and 16 for a
 *              two-qubit gate (row-major, basis ordered by (q0, q1)); may be NULL.  For a gate
 *              whose off-diagonal 2x2 blocks are exactly zero the entries of those blocks are
 *              not part of the bond decomposition and get 0.
 *   grad_params double [total gates][2]: dL/dtheta, dL/dphi of every fSim gate (0 for other
 *              kinds); may be NULL.
 *   loss       double [n_circuits]: the linear cross-entropy F of each circuit when cotangent
 *              is NULL, else NaN; may be NULL.
 * Outputs are device memory when out_on_device, else host memory; the call returns when they
 * are written.  Products run in complex64 (FP32 MFMA) whatever the grid's precision; the sum
 * over bond values and the cross-entropy are reduced in FP64.  QFLEX_E_UNSUPPORTED if a
 * qubit carries more than 64 gates. */
qflex_status qflex_contract_grad(qflex_grid* g, const uint8_t* bits, const int64_t* bs_offsets,
                                 double fidelity, uint64_t slice_seed, const int64_t* slice_ids,
                                 const int64_t* slice_offsets, const double* cotangent,
                                 int32_t cotangent_on_device, double* amps, double* grad_gates,
                                 double* grad_params, double* loss, int32_t out_on_device,
                                 void* stream);

/* Fast frugal rejection sampling over open-qubit batches (paper, Methods, "Fast sampling
 * technique"), and the sampling-error estimate of Methods, "Sampling from a non
 * fully-thermalized Porter-Thomas distribution".  All pointers are device memory; the call
 * enqueues two kernels on stream and returns (it allocates nothing).
 *   amps       complex128 [n_batch][batch_len]: row b holds batch b's amplitudes, i.e. one
 *              closed-qubit bit-string with every open-qubit value, as qflex_contract_amplitudes
 *              writes them (batch_len = 2^n_open).
 *   order      int32 [n_batch][n_c]: the open-qubit values batch b visits, in visiting order
 *              (the caller's random subset without repetition, shuffled).
 *   u          float64 [n_batch][n_c]: the uniform number in [0, 1) drawn for each visit.
 *   n_qubits   n; N = 2^n is the dimension of the Hilbert space.
 *   m          M > 0: visit j of batch b accepts its value s when u[b][j] * M < N * p, with
 *              p = re*re + im*im of amps[b][s] (each operation rounded once), i.e. with
 *              probability min(1, N p / M).  A batch stops at its first acceptance.
 *   accepted   int32 [n_batch] out: the accepted open-qubit value; -1 if none of the n_c visits
 *              accepts; -2 if a value in the batch's order row lies outside [0, batch_len)
 *              (no visit of that batch is then taken).
 *   partial    float64 [n_batch] scratch.
 *   tail       float64 [1] out: the error estimate, sum of N p over every amplitude of every
 *              batch with N p > M, divided by n_batch * batch_len (summed in FP64 in a fixed
 *              order: the same value on every run).
 * With n_batch = 0 nothing is enqueued (amps ... partial may then be NULL, tail is not
 * written).  QFLEX_E_INVALID for NULL pointers, n_batch < 0, batch_len < 1, n_c < 0,
 * n_qubits outside [1, 1000] or m <= 0 (or not finite). */
qflex_status qflex_frugal_sample(const double* amps, int64_t n_batch, int64_t batch_len,
                                 const int32_t* order, const double* u, int32_t n_c,
                                 int32_t n_qubits, double m, int32_t* accepted, double* partial,
                                 double* tail, void* stream);

/* Samples at fidelity f by the fraction of perfect-fidelity amplitudes (paper, Results,
 * "Fraction of perfect fidelity amplitudes": a sampler that returns an exact sample with
 * probability f and a uniformly random bit-string otherwise has fidelity f), each exact
 * sample drawn by frugal rejection sampling over an open-qubit batch (qflex_frugal_sample).
 * The grid must hold one circuit; all pointers are host memory.
 *   closed_bits  uint8 [n_batch][n_qubits]: batch b's closed-qubit bits (its open qubits'
 *                entries are ignored).
 *   coins        float64 [n_batch]: batch b is exact when coins[b] < fidelity (the caller's
 *                uniform draws in [0, 1)).
 *   fidelity     f in [0, 1].
 *   uniform_bits uint8 [n_batch][n_qubits]: the sample of a batch that is not exact (the
 *                caller's uniformly random bit-strings).
 *   order, u     int32 / float64 [n_batch][n_c]: visit order and uniforms of
 *                qflex_frugal_sample (rows of batches that are not exact are not read).
 *   m            M of the frugal sampler.
 *   samples      uint8 [n_batch][n_qubits] out: uniform_bits[b], or for an exact batch that
 *                accepts, closed_bits[b] with its accepted open value written into the open
 *                qubits (the first open qubit most significant).
 *   status       int8 [n_batch] out: 1 exact sample, 0 uniform sample, -1 exact batch whose
 *                n_c visits accepted nothing (its sample is then uniform_bits[b]).
 * Only the exact batches are contracted, at full fidelity, in one qflex_contract_amplitudes
 * pass; the call returns when the outputs are written.  QFLEX_E_INVALID, nothing launched, for
 * a grid of several circuits, NULL pointers, n_batch < 0, n_c < 0, fidelity outside [0, 1],
 * M <= 0 or not finite, or an order value of an exact batch outside [0, 2^n_open). */
qflex_status qflex_fidelity_samples(qflex_grid* g, const uint8_t* closed_bits, int64_t n_batch,
                                    const double* coins, double fidelity,
                                    const uint8_t* uniform_bits, const int32_t* order,
                                    const double* u, int32_t n_c, double m, uint8_t* samples,
                                    int8_t* status, void* stream);

/* The autotuner's choices (qflex_options.autotune), one table per process shared by every
 * grid: a product whose device, kind, shape and operand sources match an entry takes that
 * entry's kernel variant without being timed; every choice a grid times is added.  Saving
 * writes the table to a text file (one "<key> <variant>" line per entry, keys naming the
 * device's architecture and compute units), loading merges such a file into it (its entries
 * win), so runs that load one file pick the same kernels.  Load: *n_loaded (may be NULL)
 * receives the number of entries read; QFLEX_E_INVALID for a NULL path, a file that cannot be
 * opened or a malformed line (the table is then unchanged).  The library adds no choice
 * beyond shape rules unless a grid autotunes. */
qflex_status qflex_autotune_cache_save(const char* path);
qflex_status qflex_autotune_cache_load(const char* path, int64_t* n_loaded);
int64_t qflex_autotune_cache_size(void);
void qflex_autotune_cache_clear(void);

/* Statistics of the last contract call. */
qflex_status qflex_last_stats(const qflex_grid* g, qflex_stats* out);

/* Per-kernel timing of contract calls (tracing).  When enabled, every kernel launch of a
 * contract call is bracketed by HIP events on the call's stream; the call then waits for its
 * work to finish and adds each launch's duration to the statistics of its kernel.  Enabling
 * clears the statistics. */
typedef struct {
  char name[48];     /* kernel name, e.g. "gemm_mfma_128x128_nn", "permute" */
  int64_t launches;
  double ms;         /* summed launch durations */
  double flops;      /* algorithmic flops (8 per complex multiply-add) */
  double bytes;      /* algorithmic bytes: operands read once + result written once */
} qflex_kernel_stat;

qflex_status qflex_set_profiling(qflex_grid* g, int32_t enable);

/* Copy up to max entries of the per-kernel statistics; *n receives the number of kernels. */
qflex_status qflex_profile_read(const qflex_grid* g, qflex_kernel_stat* out, int32_t max,
                                int32_t* n);

/* Release every resource of a grid (NULL is ignored).  Waits for its work to finish. */
void qflex_grid_free(qflex_grid* g);

/* Message for the calling thread's most recent non-OK status ("" if none). */
const char* qflex_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QFLEX_H */
