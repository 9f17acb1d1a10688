"""GPU: the two kernels of a contraction step through the C ABI (qflex_permute_c64,
qflex_gemm_c64) against numpy in FP64."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_1811_09599_amd import _ffi as F

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)


def _perm_np(x, nbits, perm):
    """out[sum_j b_j 2^j] = in[sum_j b_j 2^perm[j]] via numpy.transpose on the bit axes."""
    t = x.reshape((-1,) + (2,) * nbits)  # axis 1 + i holds input bit nbits-1-i
    axes = [0] + [1 + (nbits - 1 - perm[nbits - 1 - i]) for i in range(nbits)]
    return np.transpose(t, axes).reshape(x.shape)


def _permute(x_np, nbits, perm, batch):
    torch = _torch()
    x = torch.from_numpy(x_np).cuda()
    y = torch.empty_like(x)
    p = (C.c_int32 * nbits)(*perm)
    F.check(F.lib().qflex_permute_c64(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nbits,
                                      p, batch, None))
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("nbits,batch,seed", [(1, 1, 0), (3, 2, 1), (7, 1, 2), (10, 3, 3),
                                              (12, 1, 4), (16, 2, 5), (20, 1, 6), (24, 1, 7)])
def test_permute_matches_numpy_transpose(nbits, batch, seed):
    rng = np.random.default_rng(seed)
    for trial in range(3):
        perm = list(rng.permutation(nbits)) if trial else list(range(nbits))[::-1]
        _say("permute", nbits, batch, perm)
        x = (rng.standard_normal((batch, 1 << nbits)) +
             1j * rng.standard_normal((batch, 1 << nbits))).astype(np.complex64)
        got = _permute(x, nbits, perm, batch)
        assert np.array_equal(got, _perm_np(x, nbits, perm))


def test_permute_identity_low_bits_and_worked_example():
    # Methods B.2 worked example abcdefg -> cfeadgb, each index of dimension 4 (2 bits)
    steps = [l.split() for l in open(os.path.join(GOLD, "permutation_b2.txt"))
             if l.strip() and not l.startswith("#")]
    src = steps[0][1].replace("|", "")
    dst = steps[-1][1]
    d = 2
    nbits = d * len(src)
    # label bits MSB-first: index letter i occupies bits [d*i, d*i+d) from the MSB
    in_pos = {}
    for i, ch in enumerate(src):
        for j in range(d):
            in_pos[(ch, j)] = nbits - 1 - (d * i + j)
    perm = [0] * nbits
    for i, ch in enumerate(dst):
        for j in range(d):
            perm[nbits - 1 - (d * i + j)] = in_pos[(ch, j)]
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(1 << nbits) + 1j * rng.standard_normal(1 << nbits)).astype(np.complex64)
    got = _permute(x[None], nbits, perm, 1)[0]
    want = np.transpose(x.reshape((4,) * 7), [src.index(c) for c in dst]).ravel()
    assert np.array_equal(got, want)
    # a permutation that keeps the 12 low bits in place
    perm = list(range(12)) + [15, 12, 14, 13]
    y = (rng.standard_normal((2, 1 << 16)) + 0j).astype(np.complex64)
    assert np.array_equal(_permute(y, 16, perm, 2), _perm_np(y, 16, perm))


def test_permute_rejects_bad_arguments():
    torch = _torch()
    x = torch.zeros(16, dtype=torch.complex64, device="cuda")
    p = (C.c_int32 * 4)(0, 1, 1, 3)
    st = F.lib().qflex_permute_c64(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), 4, p, 1,
                                   None)
    assert st == F.E_INVALID


def _gemm(a, b, M, N, K, ta, tb, batch, splitk=False):
    torch = _torch()
    A = torch.from_numpy(a).cuda()
    B = torch.from_numpy(b).cuda()
    Cm = torch.empty((batch, M, N), dtype=torch.complex64, device="cuda")
    L = F.lib()
    ws, ws_bytes = None, 0
    if splitk:
        ws_bytes = L.qflex_gemm_c64_workspace(M, N, K, batch)
        assert ws_bytes > 0, "shape would not be split"
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    F.check(L.qflex_gemm_c64(C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()),
                             C.c_void_p(Cm.data_ptr()), M, N, K, ta, tb, batch,
                             C.c_void_p(ws.data_ptr()) if splitk else None, ws_bytes, None))
    torch.cuda.synchronize()
    return Cm.cpu().numpy()


SHAPES = [(1, 1, 1, 1), (3, 5, 7, 2), (64, 64, 16, 1), (64, 64, 64, 3), (128, 128, 32, 1),
          (256, 128, 48, 2), (128, 256, 1024, 1), (1024, 256, 256, 1), (4096, 16, 256, 1),
          (16, 4096, 256, 1), (1 << 14, 1, 256, 2), (64, 2, 8, 5), (512, 512, 4096, 1),
          # tall-skinny rows kernel: M a multiple of 256, N <= 32, K a multiple of 16, and at
          # least 256 row blocks over the batch
          (1 << 16, 4, 256, 2), (1 << 16, 32, 64, 1), (1 << 16, 8, 16, 1), (1 << 15, 2, 64, 2),
          (3 << 15, 24, 32, 1), (1 << 16, 1, 16, 1), (1 << 16, 16, 32, 1),
          # ... on MFMA for 8 < N <= 16 (B staged 64 k at a time)
          (1 << 16, 12, 48, 1), (1 << 15, 16, 80, 2), (1 << 17, 9, 16, 1),
          # ... and its 8-deep k-tile for K = 8 (N <= 16)
          (1 << 16, 8, 8, 1), (1 << 15, 16, 8, 2), (3 << 15, 1, 8, 1), (1 << 16, 3, 8, 1),
          # reduction-shaped kernels (M <= 32, N >= 4, K >= 256; B stored [K][N]): on MFMA
          # for M <= 16 and N a multiple of 64, else on vector FMAs
          (16, 256, 1024, 2), (4, 64, 4096, 1), (32, 512, 512, 1), (1, 4, 256, 3), (3, 8, 320, 1),
          (11, 192, 512, 3), (2, 64, 256, 1),
          # short-K kernel (K < 16, N >= 32)
          (1000, 64, 4, 2), (4096, 256, 8, 1), (100, 512, 2, 3), (64, 32, 1, 1),
          # 256x128 MFMA tile (at least 256 tiles over the batch)
          (4096, 2048, 32, 1), (2048, 1024, 64, 8)]


@pytest.mark.parametrize("M,N,K,batch", SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_matches_fp64(M, N, K, batch, ta, tb):
    variant = F.lib().qflex_gemm_variant(M, N, K)
    _say("gemm", M, N, K, batch, ta, tb, "variant", variant)
    rng = np.random.default_rng(M * 7 + N * 3 + K + batch)
    sa = (batch, K, M) if ta else (batch, M, K)
    sb = (batch, N, K) if tb else (batch, K, N)
    a = (rng.standard_normal(sa) + 1j * rng.standard_normal(sa)).astype(np.complex64)
    b = (rng.standard_normal(sb) + 1j * rng.standard_normal(sb)).astype(np.complex64)
    got = _gemm(a, b, M, N, K, ta, tb, batch)
    A = a.astype(np.complex128)
    B = b.astype(np.complex128)
    if ta:
        A = np.transpose(A, (0, 2, 1))
    if tb:
        B = np.transpose(B, (0, 2, 1))
    want = A @ B
    # FP32 accumulation of K products of O(1) terms: error ~ 1e-7 * sqrt(K) relative to |C|
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < 2e-6, rel
    rms = np.sqrt(np.mean(np.abs(want) ** 2))
    assert np.max(np.abs(got - want)) < 2e-5 * rms * max(1.0, np.sqrt(K / 64))


# Reduction-shaped products (few output tiles, long K: the shapes of a gradient's operand
# cotangents) split along K into a workspace and summed in a fixed order.
SPLITK_SHAPES = [(16, 16, 1 << 16, 4, 1, 0), (4, 16, 1 << 14, 3, 1, 0), (256, 256, 8192, 1, 1, 0),
                 (64, 64, 4096, 2, 0, 0), (16, 8, 1 << 15, 2, 0, 1), (1, 1, 1 << 12, 1, 1, 1),
                 # the MFMA reduction kernel in chunks
                 (16, 256, 1 << 15, 2, 1, 0), (5, 128, 1 << 14, 3, 0, 0)]


@pytest.mark.parametrize("M,N,K,batch,ta,tb", SPLITK_SHAPES)
def test_gemm_split_k_matches_fp64_and_is_deterministic(M, N, K, batch, ta, tb):
    _say("split-K gemm", M, N, K, batch, ta, tb)
    rng = np.random.default_rng(M + 5 * N + K + batch)
    sa = (batch, K, M) if ta else (batch, M, K)
    sb = (batch, N, K) if tb else (batch, K, N)
    a = (rng.standard_normal(sa) + 1j * rng.standard_normal(sa)).astype(np.complex64)
    b = (rng.standard_normal(sb) + 1j * rng.standard_normal(sb)).astype(np.complex64)
    got = _gemm(a, b, M, N, K, ta, tb, batch, splitk=True)
    again = _gemm(a, b, M, N, K, ta, tb, batch, splitk=True)
    assert np.array_equal(got, again)
    A = np.transpose(a, (0, 2, 1)) if ta else a
    B = np.transpose(b, (0, 2, 1)) if tb else b
    want = A.astype(np.complex128) @ B.astype(np.complex128)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say("  rel", rel)
    assert rel < 2e-6, rel


SPLIT_SHAPES = [(128, 64, 16, 1), (256, 128, 64, 2), (512, 256, 256, 1), (128, 512, 1024, 1),
                (1024, 1024, 512, 1), (2048, 64, 4096, 1)]


def _split_gemm(a, b, M, N, K, ta, tb, batch, prec, tile=None):
    torch = _torch()
    A = torch.from_numpy(a).cuda()
    B = torch.from_numpy(b).cuda()
    Cm = torch.empty((batch, M, N), dtype=torch.complex64, device="cuda")
    L = F.lib()
    ws_bytes = L.qflex_gemm_split_workspace(M, N, K, batch)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    args = (C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()), C.c_void_p(Cm.data_ptr()),
            M, N, K, ta, tb, batch, F.PREC[prec], C.c_void_p(ws.data_ptr()))
    if tile is None:
        assert L.qflex_gemm_split_c64(*args, ws_bytes - 1, None) == F.E_INVALID
        F.check(L.qflex_gemm_split_c64(*args, ws_bytes, None))
    else:
        F.check(L.qflex_gemm_split_c64_tile(*args[:10], tile, args[10], ws_bytes, None))
    torch.cuda.synchronize()
    return Cm.cpu().numpy()


def _ref(a, b, ta, tb):
    A64 = a.astype(np.complex128)
    B64 = b.astype(np.complex128)
    if ta:
        A64 = np.transpose(A64, (0, 2, 1))
    if tb:
        B64 = np.transpose(B64, (0, 2, 1))
    return A64 @ B64


# bf16x3 keeps ~16 significant bits per operand: relative L2 error ~1e-5 on random data
# (measured bound 3e-5).  fp16x3 keeps ~22 bits per operand, so the FP32 accumulation
# dominates, as in the complex64 product (bound 3e-6).
SPLIT_BOUND = {"split_bf16": 3e-5, "split_fp16": 3e-6}


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("M,N,K,batch", SPLIT_SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1), (0, 1)])
def test_split_gemm_error_bound(M, N, K, batch, ta, tb, prec):
    """hi*hi + hi*lo + lo*hi per real part against the FP64 product of the same operands."""
    _say("split gemm", prec, M, N, K, batch, ta, tb)
    rng = np.random.default_rng(M + 3 * N + 7 * K + batch + 11 * ta + 13 * tb)
    sa = (batch, K, M) if ta else (batch, M, K)
    sb = (batch, N, K) if tb else (batch, K, N)
    a = (rng.standard_normal(sa) + 1j * rng.standard_normal(sa)).astype(np.complex64)
    b = (rng.standard_normal(sb) + 1j * rng.standard_normal(sb)).astype(np.complex64)
    got = _split_gemm(a, b, M, N, K, ta, tb, batch, prec)
    want = _ref(a, b, ta, tb)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say("  rel_l2", rel)
    assert rel < SPLIT_BOUND[prec], rel


# The 3-multiplication form's imaginary part P3 - P1 - P2 subtracts products whose rounding
# errors scale with |Ar + Ai| |Br + Bi|, |Ar Br| and |Ai Bi|: on random data about 1.5x the
# packed form's relative error, bounded here by twice the packed bound.
SPLIT_TILE_SIDES = {0: (256, 128), 1: (128, 128), 2: (64, 64), 3: (128, 256), 4: (256, 128),
                    5: (128, 256)}


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("tile", sorted(SPLIT_TILE_SIDES))
@pytest.mark.parametrize("M,N,K,batch,ta,tb", [(256, 256, 16, 2, 0, 0), (512, 256, 1024, 1, 1, 1),
                                              (256, 512, 256, 3, 0, 1), (1024, 256, 64, 1, 1, 0)])
def test_split_gemm_every_tile_and_form(M, N, K, batch, ta, tb, tile, prec):
    """Each output tile of the split product, packed and 3-multiplication forms, with the row
    operand gathered from complex64 (ta = 0) and pre-split (ta = 1), against FP64; one k-tile
    (K = 16) and several."""
    _say("split gemm tile", tile, prec, M, N, K, batch, ta, tb)
    rng = np.random.default_rng(M + 3 * N + 7 * K + batch + 17 * tile)
    sa = (batch, K, M) if ta else (batch, M, K)
    sb = (batch, N, K) if tb else (batch, K, N)
    a = (rng.standard_normal(sa) + 1j * rng.standard_normal(sa)).astype(np.complex64)
    b = (rng.standard_normal(sb) + 1j * rng.standard_normal(sb)).astype(np.complex64)
    got = _split_gemm(a, b, M, N, K, ta, tb, batch, prec, tile=tile)
    want = _ref(a, b, ta, tb)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    rel_re = np.linalg.norm(got.real - want.real) / np.linalg.norm(want.real)
    _say("  rel_l2", rel, "real part", rel_re)
    assert rel < SPLIT_BOUND[prec] * (2 if tile >= 4 else 1), rel
    assert rel_re < SPLIT_BOUND[prec], rel_re


def test_split_gemm_tile_entry_rejects_tiles_that_do_not_fit():
    torch = _torch()
    L = F.lib()
    M, N, K = 128, 128, 64
    A = torch.zeros((M, K), dtype=torch.complex64, device="cuda")
    B = torch.zeros((K, N), dtype=torch.complex64, device="cuda")
    Cm = torch.zeros((M, N), dtype=torch.complex64, device="cuda")
    ws_bytes = L.qflex_gemm_split_workspace(M, N, K, 1)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    P = C.c_void_p
    for tile, ok in [(-1, True), (1, True), (2, True), (0, False), (3, False), (4, False),
                     (5, False), (6, False), (-2, False)]:
        st = L.qflex_gemm_split_c64_tile(P(A.data_ptr()), P(B.data_ptr()), P(Cm.data_ptr()), M,
                                         N, K, 0, 0, 1, F.PREC["split_bf16"], tile,
                                         P(ws.data_ptr()), ws_bytes, None)
        assert (st == 0) == ok, (tile, st)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_gemm_power_of_two_scale_invariance(prec):
    """Both formats split a scaled copy exactly like the original (bf16 shares FP32's exponent
    range; fp16 takes a power-of-two scale per operand), so scaling A by 2^-70 and B by 2^50
    scales the product by exactly 2^-20, bit for bit, far outside fp16's own range."""
    M, N, K, batch = 256, 128, 256, 2
    rng = np.random.default_rng(77)
    a = (rng.standard_normal((batch, M, K)) + 1j * rng.standard_normal((batch, M, K))).astype(np.complex64)
    b = (rng.standard_normal((batch, K, N)) + 1j * rng.standard_normal((batch, K, N))).astype(np.complex64)
    c1 = _split_gemm(a, b, M, N, K, 0, 0, batch, prec)
    c2 = _split_gemm((a * np.float32(2.0 ** -70)).astype(np.complex64),
                     (b * np.float32(2.0 ** 50)).astype(np.complex64), M, N, K, 0, 0, batch, prec)
    assert np.array_equal(c2, (c1 * np.float32(2.0 ** -20)).astype(np.complex64))


def test_split_fp16_rows_of_mixed_magnitude():
    """Rows of A spread over 2^-16 .. 1 (inside the window where fp16 lo parts stay normal):
    every output row keeps the fp16x3 accuracy relative to its own size."""
    M, N, K = 256, 128, 512
    rng = np.random.default_rng(5)
    a = rng.standard_normal((1, M, K)) + 1j * rng.standard_normal((1, M, K))
    a *= 2.0 ** -rng.integers(0, 17, size=(1, M, 1))
    a = a.astype(np.complex64)
    b = (rng.standard_normal((1, K, N)) + 1j * rng.standard_normal((1, K, N))).astype(np.complex64)
    got = _split_gemm(a, b, M, N, K, 0, 0, 1, "split_fp16")
    want = _ref(a, b, 0, 0)
    row_err = np.linalg.norm(got - want, axis=2) / np.linalg.norm(want, axis=2)
    _say("  worst row", row_err.max())
    assert row_err.max() < 1e-5
