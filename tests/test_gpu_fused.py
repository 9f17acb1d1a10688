"""The fused small-plan contraction (qflex_options.fused): one launch per call, one workgroup
per bit-string running every step of the plan in LDS, against the FP64 oracle and against the
step-by-step path of the same plan."""
import ctypes as C

import numpy as np
import pytest

import rqc_inputs as R
from oracle import metrics
from oracle import slices as OS
from oracle import statevector as E1
from oracle import tn as E2
from paper_1811_09599_amd import _ffi as F
from paper_1811_09599_amd import build_grid, plan_describe

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


def _check(amps, ref, n, tol=TOL):
    e = metrics.amp_errors(amps, ref, n)
    assert e["max"] < tol, e
    return e


CASES = [
    # (rows, cols, depth, two-qubit gate, plan options, open qubits)
    (4, 4, 16, "cz", {}, []),
    (4, 4, 16, "cz", {}, [0, 5]),
    (3, 4, 8, "fsim", {}, [11]),
    (3, 3, 12, "fsim", {}, [8]),                                # 15520 LDS elements, K = 2^8
    (6, 5, 16, "cz", {}, []),                                   # 16320 of 18432 LDS elements
    (4, 4, 16, "cz", {"plan": "quadrant"}, [15]),               # 16 slices, 2 cuts
    (3, 4, 24, "cz", {"plan": "quadrant"}, []),                 # 64 slices
    (4, 4, 16, "cz", {"plan": "cut_sweep", "max_tensor_elems": 128}, []),  # 1024 slices, 5 cuts
]


@pytest.mark.parametrize("rows,cols,depth,kind,popt,op", CASES)
def test_fused_matches_state_vector_and_step_path(rows, cols, depth, kind, popt, op):
    """Every slice summed (several launches of 64 slices where there are more), with steps
    whose cuts did not change skipped: against the state vector and the step-by-step path."""
    _need_gpu()
    n = rows * cols
    _say("fused", rows, cols, depth, kind, popt, op)
    c = R.grid_rqc(rows, cols, depth, 500 + n + depth, two_qubit=kind, jitter_sd=0.02)
    bits = R.bitstrings(n, 40 if n <= 20 else 6, 7 + n, op)
    gf = build_grid(c, open_qubits=op, fused="require", **popt)
    a = gf.contract_amplitudes(bits).cpu().numpy()
    st = gf.last_stats()
    assert st["n_permute"] == 0 and st["n_slices"] == gf.num_slices(), st
    gs = build_grid(c, open_qubits=op, fused="never", **popt)
    b = gs.contract_amplitudes(bits).cpu().numpy()
    # the same products, counted the same way (steps whose cuts did not change are skipped)
    assert gs.last_stats()["flops"] == pytest.approx(st["flops"], rel=1e-12)
    # the state vector up to 20 qubits, the FP64 tensor network beyond
    ref = E1.amplitudes(c, bits, op) if n <= 20 else E2.amplitudes(c, bits, op)
    _check(a, ref, n)
    _check(a, b, n, 2e-6)


def test_fused_low_fidelity_subset_and_single_slices():
    """A seeded quarter of the slices, and single slices, against the oracle's partial sums."""
    _need_gpu()
    c = R.grid_rqc(4, 4, 16, 55)
    bits = R.bitstrings(16, 6, 2)
    g = build_grid(c, plan="quadrant", fused="require")
    S = g.num_slices()
    ids = OS.select(S, 0.25, 2700)
    a = g.contract_amplitudes(bits, fidelity=0.25, seed=2700).cpu().numpy()[:, 0]
    assert g.last_stats()["n_slices"] == len(ids)
    _check(a, E2.amplitudes(c, bits, cuts=g.plan_cuts(), slice_ids=ids), 16)
    for s in (0, S - 1):
        a = g.contract_amplitudes(bits, slice_ids=[s]).cpu().numpy()[:, 0]
        _check(a, E2.amplitudes(c, bits, cuts=g.plan_cuts(), slice_ids=[s]), 16)


def test_fused_graph_replay_and_accumulate():
    """Replays of the captured fused launch equal eager calls bit for bit, with eager work and
    synchronisation between them; accumulating calls over two halves of the slices add up to
    the call over all of them."""
    _need_gpu()
    import torch
    c = R.grid_rqc(4, 4, 16, 1001)
    sets = [R.bitstrings(16, 64, 1500), R.bitstrings(16, 64, 1501)]
    ge = build_grid(c, fused="require")
    gg = build_grid(c, fused="require", graph=True)
    for i in range(4):
        want = ge.contract_amplitudes(sets[i % 2]).cpu().numpy()
        got = gg.contract_amplitudes(sets[i % 2]).cpu().numpy()
        torch.cuda.synchronize()
        _ = torch.randn(1 << 16, device="cuda").sum().item()  # unrelated eager work
        assert np.array_equal(got, want), i
    gq = build_grid(c, plan="quadrant", fused="require")
    S = gq.num_slices()
    full = gq.contract_amplitudes(sets[0]).clone()
    out = torch.zeros_like(full)
    gq.contract_amplitudes(sets[0], slice_ids=list(range(S // 2)), out=out, accumulate=True)
    gq.contract_amplitudes(sets[0], slice_ids=list(range(S // 2, S)), out=out, accumulate=True)
    assert torch.allclose(out, full, rtol=0, atol=1e-12)


def test_fused_and_step_path_circuits_in_one_grid():
    """A grid whose circuits take different paths (one fits the fused kernel, one does not,
    as plan_describe reports beforehand)."""
    _need_gpu()
    small = R.grid_rqc(3, 3, 16, 12)
    big = R.grid_rqc(6, 6, 16, 13)  # 54336 LDS elements per bit-string: the step path
    assert plan_describe(small)["fused"]["fits"] == 1
    assert plan_describe(big)["fused"]["fits"] == 0
    bits = [R.bitstrings(9, 5, 1), R.bitstrings(36, 3, 2)]
    g = build_grid([small, big])
    g.set_profiling(True)
    a = g.contract_amplitudes(bits).cpu().numpy()[:, 0]
    prof = g.profile_read()
    g.set_profiling(False)
    assert prof["fused_contract"]["launches"] == 1 and len(prof) > 1, prof
    _check(a[:5], E1.amplitudes(small, bits[0]), 9)
    _check(a[5:], E2.amplitudes(big, bits[1]), 36)
    with pytest.raises(RuntimeError, match="does not fit"):
        build_grid(big, fused="require")


def test_fused_profile_and_stats():
    """A fused call is the only kernel work of the call (one profiled entry, whatever the
    number of 64-slice launches) and books the plan's products as the step path does."""
    _need_gpu()
    c = R.grid_rqc(4, 4, 16, 77)
    g = build_grid(c, plan="cut_sweep", max_tensor_elems=128, fused="require")
    bits = R.bitstrings(16, 3, 9)
    g.set_profiling(True)
    g.contract_amplitudes(bits)
    prof = g.profile_read()
    g.set_profiling(False)
    st = g.last_stats()
    assert set(prof) == {"fused_contract"}, prof
    assert prof["fused_contract"]["launches"] == 1, prof
    assert prof["fused_contract"]["flops"] == pytest.approx(st["flops"], rel=1e-12)
    assert st["n_slices"] == g.num_slices() == 1024 and st["n_permute"] == 0


def test_fused_more_bitstrings_than_one_launch_holds():
    """More than 65535 bit-strings: the fused contraction launches in chunks of 65535
    workgroups (one per bit-string), each chunk writing its own bit-strings' amplitudes."""
    _need_gpu()
    c = R.grid_rqc(2, 3, 8, 31)
    bits = R.bitstrings(6, 70000, 4)
    g = build_grid(c, fused="require")
    a = g.contract_amplitudes(bits).cpu().numpy()[:, 0]
    _check(a, E1.amplitudes(c, bits), 6)
    assert g.last_stats()["n_bitstrings"] == 70000


def test_fused_calls_queued_back_to_back():
    """Calls of a fused grid read their bit-strings' offsets in place from pinned host buffers
    used in turn, each rewritten only after the launches that read it two calls earlier: 12
    calls queued without any synchronisation (different bit-strings each, their own outputs)
    all equal the step path's results for the same bit-strings."""
    _need_gpu()
    import torch
    _say("fused: 12 queued calls")
    c = R.grid_rqc(4, 4, 16, 1001)
    sets = [R.bitstrings(16, 64 + 8 * i, 2600 + i) for i in range(12)]
    gs = build_grid(c, fused="never")
    want = [gs.contract_amplitudes(b).cpu().numpy() for b in sets]
    g = build_grid(c, fused="require")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        outs = [g.contract_amplitudes(b) for b in sets]
    side.synchronize()
    for i, (o, w) in enumerate(zip(outs, want)):
        e = metrics.amp_errors(o.cpu().numpy(), w, 16)
        assert e["max"] < 1e-5, (i, e)
    gs.close()
    g.close()
