// Device kernels of the contraction path and their host launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qflex {
namespace dev {

// ---------------------------------------------------------------- grid build (time collapse)
struct GridQubit {
  int32_t nlb;          // link bits of the qubit (the combo index has nlb binary digits)
  int32_t piece_begin;  // pieces [piece_begin, piece_end) in time order
  int32_t piece_end;
  int32_t pos_out;      // storage bit position (from the LSB) of the output bit
  int32_t pos_base;     // first entry in the position table (nlb entries, combo MSB first)
  int32_t pad;
  int64_t offset;       // element offset of the qubit tensor in the grid buffer
};
struct GridPiece {
  int32_t mat;    // first 2x2 matrix of the piece
  int32_t kshift; // bond digits of the piece: k = (combo >> kshift) & kmask
  int32_t kmask;
  int32_t pad;
};
void grid_build(const GridQubit* q, int n_qubits, int max_nlb, const GridPiece* pieces,
                const double2* mats, const int32_t* pos, float2* out, hipStream_t s);

// ---------------------------------------------------------------- binary index permutation
constexpr int kPermMaxTile = 10;
constexpr int kPermMaxBits = 48;
struct PermTile {
  int32_t nbits, tile_bits, nrest, pad;
  int8_t tile_in[kPermMaxTile];   // read order: bit t of i -> input bit position
  int8_t tile_out[kPermMaxTile];  // write order: bit t of j -> output bit position
  int8_t j2i[kPermMaxTile];       // bit t of j is bit j2i[t] of i
  int8_t rest_in[kPermMaxBits];   // other bits: input position
  int8_t rest_out[kPermMaxBits];  //             output position
};
// perm[j] = input bit position that feeds output bit position j (LSB = 0)
PermTile make_perm_tile(int nbits, const int* perm);
void permute(const float2* in, float2* out, int64_t batch, const PermTile& t, hipStream_t s);

// ---------------------------------------------------------------- gathered operands
// Storage positions of the bits of a product operand's row index m and of k >> 2, for an
// operand read straight from complex64 storage whose 2 lowest storage bits are k's 2 lowest
// bits: element (m, k) sits at f(m) + (k & 3) + g(k >> 2), so every group of 4 consecutive k
// is 32 contiguous bytes.
constexpr int kGatherMaxBits = 40;
constexpr int kGatherRuns = 8;
struct SplitGather {
  int32_t nm = 0, nk = 0;
  int8_t mpos[kGatherMaxBits] = {};
  int8_t kpos[kGatherMaxBits] = {};
  // Filled by gemm_split and gemm from mpos / kpos: the same maps as runs of consecutive bits
  // (bits s .. s+len-1 of m, or of the index of a tile of 16 k, land at storage positions
  // d .. d+len-1), packed as s | len << 8 | d << 16.  More than kGatherRuns runs: the kernels
  // walk the bits instead.
  int32_t nmr = 0, nkr = 0;
  int32_t mrun[kGatherRuns] = {};
  int32_t krun[kGatherRuns] = {};
};

// The same maps as runs (see SplitGather), filled on the host; returns kGatherRuns + 1 when the
// bits first .. n-1 of pos need more runs than that
int32_t gather_runs(const int8_t* pos, int first, int n, int32_t* runs);

// ---------------------------------------------------------------- complex GEMM
// C[b] = op(A[b]) * op(B[b]); A stored [M][K] (ta=0) or [K][M] (ta=1) with row stride lda,
// B stored [K][N] (tb=0) or [N][K] (tb=1) with row stride ldb, C stored [M][N].
// Batch element b starts at A + (a_off ? a_off[b] : b*a_bs) (same for B); C + b*c_bs.
// An output stored through bit-deposit maps: element (m, n) at f(m) + g(n), where f puts bit i
// of m at position mpos[i] and g bit i of n at npos[i] (one storage order of the output's
// binary labels: the positions are a permutation of 0 .. nm + nn - 1)
struct OutMap {
  int32_t nm = 0, nn = 0;
  int8_t mpos[32] = {}, npos[32] = {};
};
struct Gemm {
  const float2* A = nullptr;
  const float2* B = nullptr;
  float2* C = nullptr;
  const int64_t* a_off = nullptr;
  const int64_t* b_off = nullptr;
  int64_t a_bs = 0, b_bs = 0, c_bs = 0;
  int64_t M = 1, N = 1, K = 1;
  int64_t lda = 1, ldb = 1, ldc = 1;
  int ta = 0, tb = 0;
  int batch = 1;
  int64_t a_add = 0, b_add = 0;  // extra element offset added to every batch element
  // Split-K workspace (optional): when the product has too few output tiles to fill the GPU
  // and a long K, gemm() splits K into chunks whose partial products go to ws
  // ([chunks][batch][M][N]) and are then summed into C in a fixed order.  ws = NULL or too
  // small: no split.
  float2* ws = nullptr;
  int64_t ws_elems = 0;
  // set by gemm() for the kernels: number of K chunks and the operand offset of one chunk
  int split = 1;
  int64_t a_ks = 0, b_ks = 0;
  // kernel variant chosen by an autotuner (-1: the shape rule of gemm_variant); ignored when
  // the shape does not fit that variant
  int force_variant = -1;
  // A read straight from complex64 storage through ga (its element (m, k) at
  // f(m) + (k & 3) + g(k >> 2)) by the MFMA rows kernel, as if stored [M][K]: runs with
  // force_variant = 8 only, ta = 0, no split-K
  bool gather = false;
  SplitGather ga;
  // C written through om (the complex64 MFMA tiles and the short-K kernel: variants 1, 2, 5,
  // 6, 9 and 10, with A stored [M][K] and no split-K): element (m, n) of batch element b at
  // C + b * c_bs + f(m) + g(n); ldc unused
  bool scatter = false;
  OutMap om;
};
bool gemm_scatter_variant(int v);  // variant v can write through an OutMap
// which kernel gemm() would pick: 0 = SIMT, 1 = MFMA 64x64 tile, 2 = MFMA 128x128 tile,
// 3 = rows, 4 = reduction-shaped, 5 = short K, 6 = MFMA 256x128 tile, 7 = reduction-shaped
// on MFMA, 8 = rows on MFMA, 9 / 10 = the 256x128 / 128x128 MFMA tiles in the
// 3-multiplication form
constexpr int kGemmVariants = 11;
int gemm_variant(const Gemm& g);
bool gemm_variant_fits(const Gemm& g, int v);  // the shape meets variant v's requirements
const char* gemm_name(const Gemm& g);  // kernel name used by the profiler
// K chunks gemm() would use with an unlimited workspace, and the workspace that needs
int gemm_splitk(const Gemm& g);
int64_t gemm_splitk_elems(const Gemm& g);
void gemm(const Gemm& g, hipStream_t s);

// ---------------------------------------------------------------- split-precision products
// A complex product C = A B runs with both operands stored "K-major" ([rows][K]) in a compact
// split layout: each real part x of a complex value is split into two 16-bit values,
// hi = round(x) and lo = round(x - hi), and every group of 4 consecutive k of a row is stored
// as 16 of them
//   [rh(k0..k3), ih(k0..k3), rl(k0..k3), il(k0..k3)]            (32 bytes, 8 per complex)
// The product accumulates hi*hi + hi*lo + lo*hi of every real part in FP32 on 16-bit MFMA
// (lo*lo is dropped).  Two formats:
//  - bf16: about 16 significant bits per operand (8 + 8) over FP32's whole range;
//  - fp16: the operand is first multiplied by 2^k, chosen from its largest magnitude m so that
//    m 2^k lies in [2^14, 2^15); about 22 bits (11 + 11) for every value within 2^-17 of m,
//    fewer below (lo parts turn subnormal), and the product is multiplied back by 2^-(kA+kB).
// Permute (as permute()) into [rows][K] order, K the low kbits bits, and split.  amax = NULL
// selects bf16; otherwise fp16, with the scale taken from the slot absmax() filled.
constexpr int kSplitValues = 4;  // 16-bit values per complex element in the split layout
void split_permute(const float2* in, uint16_t* out, int64_t batch, const PermTile& t, int kbits,
                   const uint64_t* amax, hipStream_t s);
// Record max(|re|, |im|) over n complex values into *slot as (tag << 32) | float bits, by a
// 64-bit atomic maximum: the slot needs no clearing as long as every call on it uses a larger
// tag than the calls before (tag >= 1; in must be 16-byte aligned).
void absmax(const float2* in, int64_t n, uint64_t* slot, uint32_t tag, hipStream_t s);

struct GemmSplit {
  const uint16_t* A = nullptr;  // [M][K] split, row stride 4K 16-bit values
  const uint16_t* B = nullptr;  // [N][K] split
  float2* C = nullptr;          // [M][N] complex64
  const int64_t* a_off = nullptr;  // per-batch offsets in complex elements (x4 16-bit values)
  const int64_t* b_off = nullptr;
  int64_t a_bs = 0, b_bs = 0, c_bs = 0;  // batch strides: complex elements
  int64_t a_add = 0, b_add = 0;          // complex elements
  int64_t M = 0, N = 0, K = 0;
  int batch = 1;
  // fp16 operands: the absmax() slots their scales came from (both NULL: bf16 operands)
  const uint64_t* a_amax = nullptr;
  const uint64_t* b_amax = nullptr;
  // A read from complex64 storage through ga and split while staging (then A is unused and
  // a_off / a_bs / a_add count complex64 elements of Ac); NULL: A is pre-split
  const float2* Ac = nullptr;
  SplitGather ga;
  // B read from complex64 storage through gb the same way (its column index n in the place of
  // m; then B is unused and b_off / b_bs / b_add count complex64 elements of Bc); not together
  // with a gathered A
  const float2* Bc = nullptr;
  SplitGather gb;
  // output tile chosen by an autotuner: 0 = 256x128, 1 = 128x128, 2 = 64x64, 3 = 128x256, and in
  // the 3-multiplication form 4 = 256x128, 5 = 128x256 (-1 or a tile the shape does not fit: 5
  // for a gathered A where it fits, else 4, else 3 for a gathered A, else the largest of 0, 1,
  // 2 that fits)
  int tile = -1;
  // fp16 products: record the largest |re|, |im| of C into *c_amax as absmax() would, with
  // tag c_tag (NULL: not recorded)
  uint64_t* c_amax = nullptr;
  uint64_t c_tag = 0;
};
constexpr int kSplitTiles = 6;
bool gemm_split_ok(int64_t M, int64_t N, int64_t K);  // shape fits the tiled kernel
bool gemm_split_tile_fits(const GemmSplit& g, int tile);
void gemm_split(const GemmSplit& g, hipStream_t s);
const char* gemm_split_name(const GemmSplit& g);

// ---------------------------------------------------------------- fused small-plan contraction
// A whole contraction plan in one launch, one workgroup per bit-string, for plans whose
// intermediates and qubit tensors (their free parts, for the bit-string and slice) fit in the
// workgroup's LDS.  Every step is C[m][n] = sum_k X[m,k] Y[k,n] in complex64 (FP32 sums), its
// operands read in place through index tables (the bit-deposit maps of their storage orders,
// the same for every bit-string, built on the host; no permutation), C stored [M][N]; the
// result tensor is added to the FP64 amplitudes, slice after slice, with the steps whose cuts
// did not change skipped (their intermediates stay in LDS).  LDS holds the tensor image, then
// the step descriptors and index tables.
constexpr int kFusedMaxSteps = 128;
constexpr int kFusedMaxQubits = 128;
constexpr int kFusedMaxBits = 24;      // labels of one operand
constexpr int kFusedMaxKBits = 10;     // contracted labels of one step
constexpr int kFusedMaxQubitCuts = 8;  // cuts one qubit tensor depends on
constexpr int kFusedMaxCuts = 32;
constexpr int kFusedMaxSlices = 64;    // slices per launch (more: several launches)
constexpr int kFusedThreads = 1024;    // 16 waves: one bit-string's steps hide each other's latency
constexpr int64_t kFusedMaxLdsElems = 18432;  // 144 KiB of complex64 per workgroup

struct FusedQubit {
  int64_t grid_off = 0;  // the tensor in the grid (elements)
  int32_t lds = 0;       // its free part in LDS (elements)
  int32_t free_bits = 0;
  int32_t out_row = -1;  // row of the per-bit-string offsets table (closed qubits), else -1
  int32_t ncut = 0;
  int8_t cut[kFusedMaxQubitCuts] = {};    // cut index
  int8_t shift[kFusedMaxQubitCuts] = {};  // bit position of the cut's lowest label
  uint32_t deps = 0;
};
struct FusedStep {
  int32_t x = 0, y = 0, out = 0;  // LDS offsets (elements)
  int32_t mb = 0, kb = 0, nb = 0;
  uint32_t deps = 0;
  // the step's index tables (16-bit, in the plan's table block): X index of (m, k) =
  // xm[m] + xk[k], Y index of (k, n) = yk[k] + yn[n], laid out [xm | yn | xk | yk]
  int32_t tab = 0;
};
struct FusedPlan {
  const FusedStep* steps = nullptr;  // device
  const FusedQubit* qubits = nullptr;
  const uint16_t* tables = nullptr;  // every step's index tables
  int32_t nsteps = 0, nq = 0, ntab = 0;
  int32_t lds_elems = 0;  // per workgroup
  int32_t result = 0;     // LDS offset of the result tensor
  int32_t namp = 0;       // its elements
  const uint32_t* bidx = nullptr;  // result element -> open-batch index (device)
  int32_t ncut = 0;
  int8_t cut_bits[kFusedMaxCuts] = {};
};
// Contract bit-strings b0 .. b0 + nb - 1 of a circuit over `nslices` slices: offs = the
// circuit's per-bit-string offsets table ([qubit][nbs]), acc = its FP64 amplitudes
// ([bit-string][namp]), added to, or with `overwrite` set by the first slice (nslices >= 1).
void fused_setup();  // once per process and device before the first fused_contract
void fused_contract(const FusedPlan& p, const float2* grid, const int64_t* offs, int64_t nbs,
                    int64_t b0, int64_t nb, const int64_t* slices, int nslices, double2* acc,
                    bool overwrite, hipStream_t s);

// ---------------------------------------------------------------- adjoint (gradients)
constexpr int kMaxPiecesGrad = 64;  // pieces per qubit time line supported by grid_adjoint
// Cotangent of the grid build: given tbar (FP64 cotangent of every qubit tensor, laid out like
// the grid), accumulate into pbar[4*m + e] the cotangent of entry e of every 2x2 matrix m of
// the pieces (sum over all bond values of the contributions of each thread).
void grid_adjoint(const GridQubit* q, int n_qubits, int max_nlb, const GridPiece* pieces,
                  const double2* mats, const int32_t* pos, const double2* tbar, double2* pbar,
                  hipStream_t s);
// out[base + add + (off ? off[b] : 0) + o(e)] += in[b*n + e] (FP64), o(e) = the index whose
// output bit j is bit perm[j] of e; n = 2^nbits
void scatter_add_perm(const float2* in, int nbits, const int8_t* perm, int batch,
                      double2* out, const int64_t* off, int64_t add, hipStream_t s);
// dst[b*n + e] = conj(gbar[b*namp + bidx[e]]) as complex64 (seed of the reverse sweep)
void seed_cotangent(const double2* gbar, const uint32_t* bidx, int64_t n, int64_t namp,
                    int batch, float2* dst, hipStream_t s);
// gbar = scale * amps for n values; sum_sq += scale_sum * sum |amps|^2 (FP64)
void xeb_cotangent(const double2* amps, int64_t n, double scale, double2* gbar, double* sum_sq,
                   hipStream_t s);

// ---------------------------------------------------------------- reductions
// amps[b*amp_stride + bidx[e]] += res[b][e] for e < n, b < batch (FP64 accumulation)
void accumulate(const float2* res, const int64_t* r_off, int64_t r_bs, int64_t r_add, int64_t n,
                const uint32_t* bidx, double2* amps, int64_t amp_stride, int batch,
                hipStream_t s);
void fill_zero(double* p, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- sampling
// Frugal rejection sampling over open-qubit batches: accepted[b] per batch, partial[b] the
// batch's sum of N p over N p > M, *tail their sum over n_batch * batch_len (fixed order).
void frugal_sample(const double2* amps, int64_t n_batch, int64_t batch_len, const int32_t* order,
                   const double* u, int32_t n_c, int32_t n_qubits, double m, int32_t* accepted,
                   double* partial, double* tail, hipStream_t s);

}  // namespace dev
}  // namespace qflex
