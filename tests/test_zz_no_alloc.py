"""The split product without allocation (qflex_gemm_split_c64_noalloc) against the same product
on a caller's workspace (qflex_gemm_split_c64), through the C ABI: two calls in a row, the
second smaller, each equal bit for bit to the workspace call and within the split bound of the
FP64 product."""
import ctypes as C

import numpy as np
import pytest

from paper_1811_09599_amd import _ffi as F

pytestmark = pytest.mark.gpu

# relative L2 bound of one split product against FP64 (as for the workspace entry point)
SPLIT_BOUND = {"split_bf16": 3e-5, "split_fp16": 3e-6}


def _say(*a):
    print("[no_alloc]", *a, flush=True)


def _operands(M, N, K, batch, ta, tb, scale, seed):
    rng = np.random.default_rng(seed)
    sa = (batch, K, M) if ta else (batch, M, K)
    sb = (batch, N, K) if tb else (batch, K, N)
    a = (scale * (rng.standard_normal(sa) + 1j * rng.standard_normal(sa))).astype(np.complex64)
    b = (scale * (rng.standard_normal(sb) + 1j * rng.standard_normal(sb))).astype(np.complex64)
    return a, b


def _fp64(a, b, ta, tb):
    A = np.transpose(a, (0, 2, 1)) if ta else a
    B = np.transpose(b, (0, 2, 1)) if tb else b
    return A.astype(np.complex128) @ B.astype(np.complex128)


def _both(a, b, M, N, K, ta, tb, batch, prec):
    """(no-allocation result, workspace result) of the same product."""
    import torch

    L = F.lib()
    A = torch.from_numpy(a).cuda()
    B = torch.from_numpy(b).cuda()
    c_na = torch.full((batch, M, N), complex(7.0, -7.0), dtype=torch.complex64, device="cuda")
    c_ws = torch.empty((batch, M, N), dtype=torch.complex64, device="cuda")
    nws = L.qflex_gemm_split_workspace(M, N, K, batch)
    assert 0 < nws <= F.NOALLOC_SCRATCH_BYTES
    ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
    strm = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = C.c_void_p
    torch.cuda.synchronize()
    F.check(L.qflex_gemm_split_c64_noalloc(P(A.data_ptr()), P(B.data_ptr()),
                                            P(c_na.data_ptr()), M, N, K, ta, tb, batch,
                                            F.PREC[prec], strm))
    F.check(L.qflex_gemm_split_c64(P(A.data_ptr()), P(B.data_ptr()), P(c_ws.data_ptr()), M, N,
                                   K, ta, tb, batch, F.PREC[prec], P(ws.data_ptr()), nws, strm))
    torch.cuda.synchronize()
    return c_na.cpu().numpy(), c_ws.cpu().numpy()


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1), (0, 1)])
def test_noalloc_split_product_matches_workspace_entry_point(ta, tb, prec):
    # the second call is smaller and its operands 10^6 times smaller: a scale slot left over
    # from the first call would show in the fp16 result
    calls = [((1024, 512, 1024, 2), 1e3, 11), ((256, 128, 512, 1), 1e-3, 12)]
    for (M, N, K, batch), scale, seed in calls:
        _say(prec, "ta", ta, "tb", tb, "shape", (M, N, K, batch), "scale", scale)
        a, b = _operands(M, N, K, batch, ta, tb, scale, seed)
        got, want = _both(a, b, M, N, K, ta, tb, batch, prec)
        assert np.array_equal(got, want)
        ref = _fp64(a, b, ta, tb)
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say("  rel L2 vs FP64", rel)
        assert rel < SPLIT_BOUND[prec], rel
