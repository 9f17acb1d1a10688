"""GPU: graph mode (qflex_options.graph = 1).  A contract call captures its launches in a HIP
graph and later calls with the same shape replay it; every replay must equal the eager
launches bit for bit, with unrelated eager GPU work and synchronisations between replays."""
import numpy as np
import pytest

import rqc_inputs as R
from oracle import statevector as E1
from oracle import metrics
from paper_1811_09599_amd import build_grid

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precision", ["c64", "split_bf16", "split_fp16"])
def test_graph_replays_equal_eager_launches(precision):
    _need_gpu()
    import torch
    _say("graph replay,", precision)
    c = R.grid_rqc(5, 4, 24, 5151)
    op = [19, 18, 15]
    g_eager = build_grid(c, plan="quadrant", open_qubits=op, precision=precision)
    g_graph = build_grid(c, plan="quadrant", open_qubits=op, precision=precision, graph=True)
    x = torch.randn(512, 512, device="cuda")
    shapes = [4, 4, 4, 6, 4, 4]  # a new shape re-captures; returning to 4 re-captures again
    for i, nb in enumerate(shapes):
        bits = R.bitstrings(20, nb, 600 + i, op)
        want = g_eager.contract_amplitudes(bits, fidelity=0.5, seed=31).cpu().numpy()
        got = g_graph.contract_amplitudes(bits, fidelity=0.5, seed=31).cpu().numpy()
        assert np.array_equal(got, want), (i, nb)
        assert g_graph.last_stats()["flops"] == g_eager.last_stats()["flops"]
        y = x @ x  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
    # and the replayed amplitudes are right
    bits = R.bitstrings(20, 4, 700, op)
    a = g_graph.contract_amplitudes(bits).cpu().numpy()
    tol = {"c64": 1e-5, "split_bf16": 2e-4, "split_fp16": 4e-5}[precision]
    assert metrics.amp_errors(a, E1.amplitudes(c, bits, op), 20)["max"] < tol
    g_eager.close()
    g_graph.close()


def test_graph_mode_with_many_circuits():
    _need_gpu()
    _say("graph replay, 12 uneven fSim circuits")
    cs = R.fsim_batch(12, depth=12, sizes=(3, 4), seed=9100, jitter_seed0=9200)
    ge = build_grid(cs)
    gg = build_grid(cs, graph=True)
    for rep in range(3):
        bits = [R.bitstrings(c["n_qubits"], 16, 9300 + 31 * rep + i) for i, c in enumerate(cs)]
        want = ge.contract_amplitudes(bits).cpu().numpy()
        got = gg.contract_amplitudes(bits).cpu().numpy()
        assert np.array_equal(got, want), rep


def test_graph_mode_on_the_callers_stream():
    """A grid in graph mode captures and replays on a caller's stream that is not the null
    stream (no stream of its own in between); replays equal eager launches bit for bit."""
    _need_gpu()
    import torch
    _say("graph replay on a side stream")
    c = R.grid_rqc(4, 4, 16, 1001)
    # the step path: a call of fused circuits is launched directly, not captured
    ge = build_grid(c, fused="never")
    gg = build_grid(c, graph=True, fused="never")
    side = torch.cuda.Stream()
    for rep in range(4):
        bits = R.bitstrings(16, 64, 1500 + rep)
        want = ge.contract_amplitudes(bits).cpu().numpy()
        with torch.cuda.stream(side):
            got = gg.contract_amplitudes(bits)
        side.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), rep
    ge.close()
    gg.close()


def test_graph_mode_launches_fused_calls_directly():
    """A call whose circuits all run the fused small-plan kernel is one launch per circuit: in
    graph mode it is launched directly (its launches show in the profile, which a capture
    would switch off), with the eager grid's results; a grid that also holds a circuit on the
    step path still captures and replays."""
    _need_gpu()
    _say("graph mode, fused calls")
    c = R.grid_rqc(4, 4, 16, 1001)
    ge = build_grid(c)
    gg = build_grid(c, graph=True)
    gg.set_profiling(True)
    for rep in range(3):
        bits = R.bitstrings(16, 64, 1600 + rep)
        want = ge.contract_amplitudes(bits).cpu().numpy()
        got = gg.contract_amplitudes(bits).cpu().numpy()
        assert np.array_equal(got, want), rep
    prof = gg.profile_read()
    gg.set_profiling(False)
    assert prof["fused_contract"]["launches"] == 3, prof
    ge.close()
    gg.close()
    # mixed: captured by the first call, replayed by the later ones (no profiled launches)
    small, big = R.grid_rqc(3, 3, 16, 12), R.grid_rqc(6, 6, 16, 13)
    ge = build_grid([small, big])
    gg = build_grid([small, big], graph=True)
    for rep in range(3):
        bits = [R.bitstrings(9, 4, 1700 + rep), R.bitstrings(36, 2, 1800 + rep)]
        want = ge.contract_amplitudes(bits).cpu().numpy()
        if rep == 2:
            gg.set_profiling(True)
        got = gg.contract_amplitudes(bits).cpu().numpy()
        assert np.array_equal(got, want), rep
    prof = gg.profile_read()
    gg.set_profiling(False)
    assert "fused_contract" not in prof, prof
    ge.close()
    gg.close()


@pytest.mark.parametrize("side_stream", [False, True])
def test_gradient_graph_replays_match_eager(side_stream):
    """qflex_contract_grad in graph mode (one slice per circuit: 10 uneven fSim circuits, no
    cuts): the first call captures, later calls with new bit-strings and cotangents replay.
    Amplitudes equal the eager call's bit for bit; gradients and cross-entropies agree to
    1e-12 (their FP64 sums are atomic, so their order may differ)."""
    _need_gpu()
    import torch
    _say("gradient graph replay, side stream:", side_stream)
    cs = R.fsim_batch(10, depth=12, sizes=(3, 4), seed=9400, jitter_seed0=9500)
    ge = build_grid(cs)
    gg = build_grid(cs, graph=True)
    side = torch.cuda.Stream() if side_stream else None
    x = torch.randn(256, 256, device="cuda")
    rng = np.random.default_rng(9)
    for rep in range(4):
        bits = [R.bitstrings(c["n_qubits"], 12, 9600 + 17 * rep + i) for i, c in enumerate(cs)]
        cot = None
        if rep == 3:  # a given cotangent: a graph of its own
            cot = rng.standard_normal((120, 1)) + 1j * rng.standard_normal((120, 1))
        want = ge.contract_grad(bits, cotangent=cot)
        if side is not None:
            with torch.cuda.stream(side):
                got = gg.contract_grad(bits, cotangent=cot)
            side.synchronize()
        else:
            got = gg.contract_grad(bits, cotangent=cot)
        assert np.array_equal(np.asarray(got["amps"]), np.asarray(want["amps"])), rep
        for i in range(len(cs)):
            gw, gr = np.asarray(want["grad_params"][i]), np.asarray(got["grad_params"][i])
            assert np.linalg.norm(gr - gw) <= 1e-12 * max(np.linalg.norm(gw), 1e-300), (rep, i)
        if cot is None:
            assert np.allclose(got["loss"], want["loss"], rtol=1e-12, atol=1e-14), rep
        y = x @ x  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
    ge.close()
    gg.close()
