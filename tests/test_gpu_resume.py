"""GPU: the slices of one amplitude batch spread over several accumulating calls
(QFLEX_OUT_ACCUMULATE) equal one call over all of them, bit for bit.  Intermediates that depend
on no cut whose value changed are kept across the calls, as across the slices of one call
(SI A reuse), so the chain does the work of the single call and no more."""
import ctypes as C

import numpy as np
import pytest

import rqc_inputs as R
from oracle import metrics
from oracle import statevector as E1
from paper_1811_09599_amd import _ffi as F
from paper_1811_09599_amd import build_grid

pytestmark = pytest.mark.gpu
OPEN7 = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
TOL = {"c64": 1e-5, "split_bf16": 2e-4, "split_fp16": 4e-5}


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


def _chain(g, bits, ids, out):
    flops = []
    for s in ids:
        g.contract_amplitudes(bits, slice_ids=[s], out=out, accumulate=True)
        flops.append(g.last_stats()["flops"])
    return flops


@pytest.mark.parametrize("prec", ["c64", "split_bf16", "split_fp16"])
def test_accumulating_single_slice_calls_equal_one_call(prec):
    import torch
    _need_gpu()
    _say("4x5 depth 24 quadrant, slices over accumulating calls,", prec)
    c = R.grid_rqc(4, 5, 24, 320)
    op = [19, 18, 14]
    bits = R.bitstrings(20, 3, 8, op)
    other = R.bitstrings(20, 3, 9, op)
    g = build_grid(c, plan="quadrant", open_qubits=op, precision=prec)
    S = g.num_slices()
    assert S > 4 and len(g.plan_cuts()) == 2
    full = g.contract_amplitudes(bits)
    f_full = g.last_stats()["flops"]
    g.contract_amplitudes(other)  # the arena now holds other bit-strings: nothing to reuse
    out = torch.zeros_like(full)
    flops = _chain(g, bits, range(S), out)
    assert torch.equal(out, full)
    # the first call runs every step, the later ones only what their changed cuts touch
    assert sum(flops) == f_full and flops[0] > flops[1]
    e = metrics.amp_errors(out.cpu().numpy(), E1.amplitudes(c, bits, op), 20)
    assert e["max"] < TOL[prec], e
    # different bit-strings after the chain: nothing reused, the result as on a fresh grid
    g.contract_amplitudes(other, slice_ids=[3])
    assert g.last_stats()["flops"] == flops[0]
    fresh = build_grid(c, plan="quadrant", open_qubits=op, precision=prec)
    assert torch.equal(g.contract_amplitudes(other, slice_ids=[3]),
                       fresh.contract_amplitudes(other, slice_ids=[3]))
    g.close()
    fresh.close()


@pytest.mark.parametrize("opts", [{"bitstring_batch": 2}, {"graph": True}])
def test_accumulating_calls_without_reuse_still_equal_one_call(opts):
    """Several batches per call (the arena then holds the last one, not the first) and graph
    mode (which keeps nothing across calls): the chain recomputes and still sums the same."""
    import torch
    _need_gpu()
    _say("4x5 depth 24, accumulating calls,", opts)
    c = R.grid_rqc(4, 5, 24, 320)
    op = [19, 18, 14]
    bits = R.bitstrings(20, 3, 8, op)
    g = build_grid(c, plan="quadrant", open_qubits=op, **opts)
    S = g.num_slices()
    full = g.contract_amplitudes(bits)
    f_full = g.last_stats()["flops"]
    out = torch.zeros_like(full)
    flops = _chain(g, bits, range(S), out)
    assert torch.equal(out, full)
    assert flops[1] == flops[0] and sum(flops) > f_full
    g.close()


@pytest.mark.parametrize("prec", ["c64", "split_bf16"])
def test_7x7_block_subset_over_calls_equals_one_call(prec):
    """The bench's pattern at bond dimension 16: one bit-string, the slices of a block subset
    (one right-cut value, consecutive bottom-cut values) one per accumulating call."""
    import torch
    _need_gpu()
    _say("7x7 depth 1+32+1 block subset over calls,", prec)
    c = R.grid_rqc(7, 7, 32, 2000)
    bits = R.bitstrings(49, 2, 2500, OPEN7)[:1]
    g = build_grid(c, open_qubits=OPEN7, precision=prec, slice_mode="block")
    ids = list(range(16 * 5, 16 * 5 + 6))
    one = g.contract_amplitudes(bits, slice_ids=ids)
    f_one = g.last_stats()["flops"]
    g.contract_amplitudes(R.bitstrings(49, 1, 2600, OPEN7), slice_ids=[0])
    out = torch.zeros_like(one)
    flops = _chain(g, bits, ids, out)
    assert torch.equal(out, one)
    assert sum(flops) == f_one
    g.close()


def test_output_flags_are_checked():
    import torch
    _need_gpu()
    c = R.grid_rqc(3, 3, 8, 5)
    bits = R.bitstrings(9, 2, 1)
    g = build_grid(c)
    out = torch.zeros((2, 1), dtype=torch.complex128, device="cuda")
    L = F.lib()
    offs = np.array([0, 2], dtype=np.int64)
    flat = np.ascontiguousarray(bits.ravel())
    for flags in (2, 4, -1):
        st = L.qflex_contract_amplitudes(g._h, flat.ctypes.data_as(C.POINTER(C.c_uint8)),
                                         offs.ctypes.data_as(C.POINTER(C.c_int64)), 1.0,
                                         C.c_uint64(0), None, None, C.c_void_p(out.data_ptr()),
                                         flags, C.c_void_p(0))
        assert st == F.E_INVALID, flags
    with pytest.raises(ValueError):
        g.contract_amplitudes(bits, accumulate=True)
    # accumulating twice doubles
    ref = g.contract_amplitudes(bits)
    g.contract_amplitudes(bits, out=out, accumulate=True)
    g.contract_amplitudes(bits, out=out, accumulate=True)
    assert torch.equal(out, 2 * ref)
    g.close()


def test_resume_reads_each_circuits_own_rows():
    """A call resumes a batch only when its bit-strings equal the kept batch's, read from the
    circuit's own rows of the concatenated input (each circuit's rows are its own width).
    Here circuit 0 (30 qubits, fused kernel) keeps its bit-strings between two calls and
    circuit 1 (20 qubits, step path, whose last batch is the one kept) changes them; reading
    circuit 1's rows at 20 bytes per earlier row would compare bytes of circuit 0 instead
    (equal in both calls) and return the first call's amplitudes."""
    _need_gpu()
    _say("resume: rows of circuits of different widths")
    c0, c1 = R.grid_rqc(6, 5, 16, 21), R.grid_rqc(4, 5, 24, 22)
    g = build_grid([c0, c1])
    b0 = R.bitstrings(30, 4, 2301)
    first = g.contract_amplitudes([b0, R.bitstrings(20, 2, 2302)]).cpu().numpy()[:, 0]
    b1 = R.bitstrings(20, 2, 2303)
    second = g.contract_amplitudes([b0, b1]).cpu().numpy()[:, 0]
    assert metrics.amp_errors(second[4:], E1.amplitudes(c1, b1), 20)["max"] < TOL["c64"]
    assert np.array_equal(second[:4], first[:4])  # circuit 0: same bit-strings, same kernel
    g.close()


@pytest.mark.parametrize("graph", [False, True])
def test_heterogeneous_grid_over_calls(graph):
    """One grid of circuits of 9, 20, 6 and 16 qubits (the 9- and 6-qubit ones on the fused
    kernel, the others on the step path), called repeatedly with bit-string counts that
    include 0 and with some circuits' bit-strings kept and others changed from one call to the
    next: every call's amplitudes match the state vector, in eager and in graph mode."""
    _need_gpu()
    _say("heterogeneous grid over calls, graph:", graph)
    cs = [R.grid_rqc(3, 3, 12, 31, two_qubit="fsim"), R.grid_rqc(4, 5, 24, 32),
          R.grid_rqc(2, 3, 8, 33), R.grid_rqc(4, 4, 20, 34)]
    g = build_grid(cs, graph=graph)
    counts = [[3, 2, 0, 4], [3, 2, 0, 4], [0, 2, 5, 1], [3, 2, 0, 4], [3, 2, 0, 4]]
    seeds = [[1, 2, 3, 4], [1, 5, 3, 4], [6, 7, 8, 9], [1, 7, 3, 10], [11, 7, 3, 10]]
    for call, (cnt, sd) in enumerate(zip(counts, seeds)):
        bits = [R.bitstrings(c["n_qubits"], m, 2400 + s) for c, m, s in zip(cs, cnt, sd)]
        got = g.contract_amplitudes(bits).cpu().numpy()[:, 0]
        at = 0
        for c, b in zip(cs, bits):
            m = len(b)
            if m:
                e = metrics.amp_errors(got[at:at + m], E1.amplitudes(c, b), c["n_qubits"])
                assert e["max"] < TOL["c64"], (call, c["n_qubits"], e)
            at += m
        assert at == len(got)
    g.close()
