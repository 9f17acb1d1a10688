/*
 * qflex_kernels.h - the two kernels of every pairwise contraction step of libqflex, exposed on
 * their own (paper, Methods B.2: an index permutation that makes the contracted indexes
 * contiguous, then a matrix multiplication), plus the seeded slice subset of Methods C.1.
 *
 * Pointers marked "device" are HIP device memory owned by the caller; complex64 values are
 * interleaved (re, im) floats.  Every call checks its arguments on the host before launching
 * and returns QFLEX_E_INVALID without launching anything when they are wrong.  Work is
 * enqueued on `stream` (a hipStream_t, NULL = null stream) and is not waited for.
 */
#ifndef QFLEX_KERNELS_H
#define QFLEX_KERNELS_H

#include <stdint.h>

#include "qflex.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Permute the binary indexes of `batch` tensors of 2^nbits complex64 elements each
 * (row-major, batch-major, device).  perm[j] (j = 0 .. nbits-1, counted from the least
 * significant bit) is the input bit position that becomes output bit position j:
 * out[sum_j b_j 2^j] = in[sum_j b_j 2^perm[j]].  1 <= nbits <= 40, perm a permutation,
 * 1 <= batch <= 65535, in and out must not overlap. */
qflex_status qflex_permute_c64(const void* in, void* out, int32_t nbits, const int32_t* perm,
                               int64_t batch, void* stream);

/* Batched complex64 matrix product C[b] = op(A[b]) op(B[b]) with FP32 accumulation (device).
 * A[b] is stored [M][K] (ta = 0) or [K][M] (ta = 1), B[b] is [K][N] (tb = 0) or [N][K]
 * (tb = 1), C[b] is [M][N]; all row-major and densely packed, batch b at offset b*size.
 * M, N, K >= 1, 1 <= batch <= 65535.  C must not overlap A or B.
 * workspace (optional, device, NULL allowed): when it holds at least
 * qflex_gemm_c64_workspace(M, N, K, batch) bytes and that is non-zero, a product with few
 * output tiles and a long K is split along K; the partial products land in the workspace and
 * are summed into C in a fixed order (same result on every run).  Otherwise, or with
 * workspace = NULL, the product runs unsplit.  The call allocates nothing itself. */
qflex_status qflex_gemm_c64(const void* A, const void* B, void* C, int64_t M, int64_t N,
                            int64_t K, int32_t ta, int32_t tb, int64_t batch, void* workspace,
                            int64_t workspace_bytes, void* stream);
int64_t qflex_gemm_c64_workspace(int64_t M, int64_t N, int64_t K, int64_t batch);

/* The same product in split precision: each real part x of a complex64 operand is split into
 * two 16-bit parts, hi = round(x) and lo = round(x - hi); the three products hi*hi + hi*lo +
 * lo*hi run on 16-bit MFMA with FP32 accumulation (lo*lo is dropped).  The complex product
 * takes the 3-multiplication form (see qflex_gemm_split_c64_tile) where its tiles fit (M a
 * multiple of 256 and N of 128, or of 128 and 256), else the packed form.
 *   precision = QFLEX_PREC_SPLIT_BF16: bf16 parts, about 16 significant bits per operand.
 *   precision = QFLEX_PREC_SPLIT_FP16: fp16 parts of the operand times 2^k, k chosen from the
 *     operand's largest magnitude m (over the whole batch) so that m 2^k is in [2^14, 2^15);
 *     about 22 significant bits for values within 2^-17 of m, fewer below; the result is
 *     scaled back by 2^-(kA+kB).
 * (Split-precision products are not in the paper, which multiplies in complex64.)
 * M, N, K must be powers of two, multiples of 64 (M, N) and 16 (K); A and B 16-byte aligned.
 * workspace: device memory, 16-byte aligned, of at least qflex_gemm_split_workspace(M, N, K,
 * batch) bytes, used for the split operands and the two scale slots (the call allocates
 * nothing itself; calls sharing one workspace must be ordered on one stream). */
qflex_status qflex_gemm_split_c64(const void* A, const void* B, void* C, int64_t M, int64_t N,
                                  int64_t K, int32_t ta, int32_t tb, int64_t batch,
                                  int32_t precision, void* workspace, int64_t workspace_bytes,
                                  void* stream);
int64_t qflex_gemm_split_workspace(int64_t M, int64_t N, int64_t K, int64_t batch);

/* qflex_gemm_split_c64 with the kernel's output tile and complex form chosen by the caller (an
 * autotuner's candidates).  The packed form computes Re C and Im C each as one real product over
 * 2K terms ([Ar Ai].[Br; -Bi] and [Ar Ai].[Bi; Br]: 12 16-bit MFMAs per 32x32 block and 16
 * complex k); the 3-multiplication (Gauss) form computes P1 = Ar.Br, P2 = Ai.Bi and
 * P3 = (Ar + Ai).(Br + Bi) and takes Re C = P1 - P2, Im C = P3 - P1 - P2 (9 MFMAs; Im C's error
 * grows with |Ar + Ai| |Br + Bi| + |Ar Br| + |Ai Bi| rather than with |A| |B|).
 *   tile = 0: 256x128, 1: 128x128, 2: 64x64, 3: 128x256, packed form;
 *          4: 256x128, 5: 128x256, 3-multiplication form;
 *         -1: the choice qflex_gemm_split_c64 makes.
 * QFLEX_E_INVALID, nothing launched, for any other tile or one M, N do not fit (multiples of the
 * tile's sides); every other argument and error as qflex_gemm_split_c64. */
qflex_status qflex_gemm_split_c64_tile(const void* A, const void* B, void* C, int64_t M,
                                       int64_t N, int64_t K, int32_t ta, int32_t tb,
                                       int64_t batch, int32_t precision, int32_t tile,
                                       void* workspace, int64_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): qflex_gemm_split_c64 with its workspace taken from a
 * static device buffer of the library, QFLEX_NOALLOC_SCRATCH_BYTES per GPU, held by every GPU
 * the library is loaded on until the process ends.  Arguments, layouts, checks and results are
 * those of qflex_gemm_split_c64 (the same kernels, bit for bit); A, B and C stay the caller's.
 * The call allocates and frees nothing: on its first call on a device (the current one) it
 * looks up that device's copy of the buffer, then only enqueues kernels on `stream`; the fp16
 * scale slots are cleared by a fill kernel on every call.
 * QFLEX_E_INVALID, nothing launched, when qflex_gemm_split_workspace(M, N, K, batch) exceeds
 * QFLEX_NOALLOC_SCRATCH_BYTES.  Every call on one GPU shares that GPU's buffer: calls that
 * may overlap on one GPU (different streams without ordering, or different threads) race and
 * give wrong results; calls ordered on one stream are safe.  `stream` must belong to the
 * current device. */
#define QFLEX_NOALLOC_SCRATCH_BYTES (64ll << 20)
qflex_status qflex_gemm_split_c64_noalloc(const void* A, const void* B, void* C, int64_t M,
                                          int64_t N, int64_t K, int32_t ta, int32_t tb,
                                          int64_t batch, int32_t precision, void* stream);

/* Kernel variant qflex_gemm_c64 uses for a shape: 0 SIMT, 1 MFMA 64x64, 2 MFMA 128x128,
 * 3 tall-skinny rows kernel (M a multiple of 256 and at least 32768, N <= 32, K a multiple
 * of 16, or K = 8 with N <= 16), 4 reduction kernel (M <= 32, N >= 4 a power of two or a
 * multiple of 256, K >= 256 a multiple of 64, B not transposed), 5 short-K kernel (K < 16 a
 * power of two, N >= 32 as in 4), 6 MFMA 256x128 (M a multiple of 256, N of 128, K of 16, and
 * at least 256 such tiles over the batch), 7 reduction kernel on MFMA (M <= 16, N a multiple
 * of 64, K >= 256 a multiple of 64, B not transposed; picked before 4), 8 rows kernel on MFMA
 * (as 3 with K a multiple of 16 and N <= 16; picked before 3 when N > 8), 9 and 10 the
 * 256x128 and 128x128 MFMA tiles in the 3-multiplication (Gauss) form: P1 = Ar Br, P2 = Ai Bi,
 * P3 = (Ar + Ai)(Br + Bi), C = (P1 - P2) + i (P3 - P1 - P2), three real products instead of
 * four, picked in place of 6 and 2.  This query assumes batch = 1. */
int32_t qflex_gemm_variant(int64_t M, int64_t N, int64_t K);

/* The slice subset that qflex_contract_amplitudes sums for a fidelity (host only): writes up to
 * max_ids ascending ids into ids and their count into *n.  mode: qflex_slice_mode.
 * QFLEX_E_INVALID if fidelity is outside (0, 1] or mode is unknown, QFLEX_E_PLAN if
 * fidelity*total is not an integer >= 1 (or, in block mode, does not divide total). */
qflex_status qflex_select_slices(int64_t total, double fidelity, uint64_t seed, int32_t mode,
                                 int64_t* ids, int64_t max_ids, int64_t* n);

#ifdef __cplusplus
}
#endif

#endif /* QFLEX_KERNELS_H */
