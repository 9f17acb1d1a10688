"""GPU: adjoint contraction (qflex_contract_grad) against the FP64 oracle's gradients, to 1e-3
relative L2 per circuit."""
import numpy as np
import pytest

import rqc_inputs as R
from oracle import gates as G
from oracle import metrics
from oracle import statevector as E1
from oracle import tn as E2
from paper_1811_09599_amd import build_grid

pytestmark = pytest.mark.gpu
GTOL = 1e-3


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


def _fsim_rows(c):
    return [i for i, g in enumerate(c["gates"]) if g["kind"] == "fsim"]


@pytest.mark.parametrize("rows,cols,plan", [(3, 3, "auto"), (3, 4, "auto"), (4, 4, "auto"),
                                            (4, 4, "quadrant"), (2, 5, "auto")])
def test_linear_xeb_gradient_vs_state_vector_adjoint(rows, cols, plan):
    _need_gpu()
    _say("xeb grad", rows, cols, plan)
    n = rows * cols
    c = R.grid_rqc(rows, cols, 12, 500 + n, two_qubit="fsim", jitter_sd=0.02, jitter_seed=7 + n)
    bits = R.bitstrings(n, 24, 31 + n)
    g = build_grid(c, plan=plan)
    res = g.contract_grad(bits)
    f_ref, g_ref = E1.linear_xeb_grad(c, bits)
    got = res["grad_params"][0][_fsim_rows(c)]
    err = metrics.rel_l2(got, g_ref)
    _say("  rel err", err, "loss", res["loss"][0], f_ref)
    assert err < GTOL
    assert abs(res["loss"][0] - f_ref) < 1e-4 * max(1.0, abs(f_ref))
    assert metrics.amp_errors(res["amps"][:, 0], E1.amplitudes(c, bits), n)["max"] < 1e-5


def test_custom_cotangent_and_gate_entry_gradients():
    _need_gpu()
    _say("custom cotangent")
    c = R.grid_rqc(3, 4, 12, 77, two_qubit="fsim", jitter_sd=0.02, jitter_seed=3)
    bits = R.bitstrings(12, 10, 5)
    rng = np.random.default_rng(1)
    cot = rng.standard_normal(10) + 1j * rng.standard_normal(10)
    res = build_grid(c).contract_grad(bits, cotangent=cot[:, None])
    assert np.isnan(res["loss"][0])
    # cot = dL/dRe psi + i dL/dIm psi, so dL/dtheta = Re sum conj(cot) dpsi/dtheta
    dth, dph, psi = E1.vjp_params(c, bits, np.conj(cot))
    ref = np.stack([dth.real, dph.real], axis=1)
    got = res["grad_params"][0][_fsim_rows(c)]
    assert metrics.rel_l2(got, ref) < GTOL
    # gate entries: dL/dRe G + i dL/dIm G = conj(sum_b conj(cot_b) dpsi_b/dG)
    dgate = E1.vjp_gates(c, bits, np.conj(cot))
    target = np.sum(np.conj(cot) * psi)
    for i, gt in enumerate(c["gates"]):
        gg = res["grad_gates"][0][i]
        mat = G.matrix(gt)
        # Euler identity: psi is linear in each gate's entries
        assert abs(np.sum(np.conj(gg) * mat) - target) < 1e-3 * abs(target) + 1e-9, i
        if gt["kind"] != "cz":  # every entry of a rank-4 or one-qubit gate is in the bonds
            assert metrics.rel_l2(np.conj(gg), dgate[i]) < GTOL, i


def test_uneven_circuits_in_one_call():
    _need_gpu()
    _say("uneven batch grad")
    cs = R.fsim_batch(5, depth=12, sizes=(3, 4), seed=8000, jitter_seed0=8100)
    bits = [R.bitstrings(c["n_qubits"], 12 + 2 * i, 300 + i) for i, c in enumerate(cs)]
    res = build_grid(cs).contract_grad(bits)
    for i, c in enumerate(cs):
        f_ref, g_ref = E1.linear_xeb_grad(c, bits[i])
        got = res["grad_params"][i][_fsim_rows(c)]
        assert metrics.rel_l2(got, g_ref) < GTOL, i
        assert abs(res["loss"][i] - f_ref) < 1e-4 * max(1.0, abs(f_ref)), i


def test_uneven_circuits_with_several_slices():
    """Circuits of 16, 12 and 9 qubits in one grid, each summing its own subset of several
    slices (the amplitudes first, through the contraction path of each circuit: the 9-qubit one
    on the fused kernel; then one reverse sweep per slice), an open qubit and a given
    cotangent: every circuit's angle gradients and amplitudes against the FP64 network's."""
    _need_gpu()
    _say("uneven circuits, several slices each")
    cs = [R.grid_rqc(4, 4, 12, 31, two_qubit="fsim", jitter_sd=0.02, jitter_seed=31),
          R.grid_rqc(3, 4, 12, 32, two_qubit="fsim", jitter_sd=0.02, jitter_seed=32),
          R.grid_rqc(3, 3, 12, 33, two_qubit="fsim", jitter_sd=0.02, jitter_seed=33)]
    op = [0]
    bits = [R.bitstrings(c["n_qubits"], m, 3100 + i, op) for i, (c, m) in enumerate(zip(cs, (3, 4, 2)))]
    g = build_grid(cs, plan="quadrant", open_qubits=op)
    ids = [[0, 7, 100, 255], [1, 9, 15], [3, 128]]
    assert [g.num_slices(i) for i in range(3)] == [256, 16, 256]
    rng = np.random.default_rng(31)
    cot = rng.standard_normal((9, 2)) + 1j * rng.standard_normal((9, 2))
    res = g.contract_grad(bits, cotangent=cot, slice_ids=ids)
    at = 0
    for i, c in enumerate(cs):
        m = len(bits[i])
        cuts = g.plan_cuts(i)
        ref = E2.amplitude_gate_grads(c, bits[i], cot[at:at + m], op, cuts, ids[i])
        got = res["grad_params"][i][_fsim_rows(c)]
        assert metrics.rel_l2(got, ref) < GTOL, i
        amp_ref = E2.amplitudes(c, bits[i], op, cuts=cuts, slice_ids=ids[i])
        assert metrics.amp_errors(res["amps"][at:at + m], amp_ref, c["n_qubits"])["max"] < 1e-5, i
        at += m
    g.close()


@pytest.mark.parametrize("one_slice", [False, True])
def test_gradient_with_open_batch_and_fidelity_subset(one_slice):
    """Several slices (amplitudes first, then one reverse sweep per slice) and a single slice
    (the forward pass of the reverse sweep also yields the amplitudes)."""
    _need_gpu()
    _say("open batch + fidelity subset grad, one slice:", one_slice)
    c = R.grid_rqc(4, 4, 12, 909, two_qubit="fsim", jitter_sd=0.02, jitter_seed=12)
    op = [15, 14]
    bits = R.bitstrings(16, 6, 2, op)
    g = build_grid(c, plan="quadrant", open_qubits=op)
    S = g.num_slices()
    ids = [5] if one_slice else [0, 5, S // 2, S - 1]
    rng = np.random.default_rng(3)
    cot = rng.standard_normal((6, 4)) + 1j * rng.standard_normal((6, 4))
    res = g.contract_grad(bits, cotangent=cot, slice_ids=ids)
    cuts = g.plan_cuts()
    ref = E2.amplitude_gate_grads(c, bits, cot, op, cuts, ids)
    got = res["grad_params"][0][_fsim_rows(c)]
    assert metrics.rel_l2(got, ref) < GTOL
    amp_ref = E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=ids)
    assert metrics.amp_errors(res["amps"], amp_ref, 16)["max"] < 1e-5


def test_6x6_gradient_vs_autograd_oracle():
    _need_gpu()
    _say("6x6 fSim grad vs E3")
    c = R.grid_rqc(6, 6, 12, 6600, two_qubit="fsim", jitter_sd=0.02, jitter_seed=66)
    bits = R.bitstrings(36, 3, 36)
    res = build_grid(c).contract_grad(bits)
    f_ref, g_ref = E2.linear_xeb_grad(c, bits)
    got = res["grad_params"][0][_fsim_rows(c)]
    assert metrics.rel_l2(got, g_ref) < GTOL
    assert abs(res["loss"][0] - f_ref) < 1e-4 * max(1.0, abs(f_ref))


def test_7x7_one_slice_gradient_vs_autograd_oracle():
    """7x7 fSim depth 1+16+1 (bond 16): the quadrant plan with two cuts, one slice, a 64-amplitude
    open batch and a random cotangent.  The adjoint keeps only its checkpoints (the plan's
    gradient layout has several segments, each recomputed before it is reversed) and matches
    the FP64 autograd oracle on that slice."""
    from paper_1811_09599_amd import plan_describe

    _need_gpu()
    _say("7x7 fSim one-slice grad vs E3")
    c = R.grid_rqc(7, 7, 16, 7700, two_qubit="fsim", jitter_sd=0.02, jitter_seed=77)
    op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    lay = plan_describe(c, open_qubits=op)["grad"]
    assert len(lay["segments"]) >= 2 and lay["recompute_flops"] > 0
    assert 2 * lay["elems"] < lay["store_all_elems"]
    bits = R.bitstrings(49, 1, 7701, op)
    rng = np.random.default_rng(5)
    cot = rng.standard_normal((1, 64)) + 1j * rng.standard_normal((1, 64))
    g = build_grid(c, open_qubits=op)
    res = g.contract_grad(bits, cotangent=cot, slice_ids=[37])
    cuts = g.plan_cuts()
    order = E2.quadrant_order(7, 7)
    ref = E2.amplitude_gate_grads(c, bits, cot, op, cuts, [37], order=order)
    got = res["grad_params"][0][_fsim_rows(c)]
    err = metrics.rel_l2(got, ref)
    _say("  rel err", err)
    assert err < GTOL
    amp_ref = E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=[37], order=order)
    assert metrics.amp_errors(res["amps"], amp_ref, 49)["max"] < 1e-5


def test_autograd_function_fits_angles():
    _need_gpu()
    import torch
    from paper_1811_09599_amd import Amplitudes
    _say("autograd")
    c = R.grid_rqc(3, 3, 12, 4242, two_qubit="fsim", jitter_sd=0.02, jitter_seed=42)
    bits = R.bitstrings(9, 16, 9)
    p0 = R.fsim_params(c)
    ang = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    amps = Amplitudes.apply(ang, c, bits)
    f = (2.0 ** 9) * torch.mean(amps.abs() ** 2) - 1.0
    f.backward()
    f_ref, g_ref = E1.linear_xeb_grad(c, bits)
    assert abs(float(f.detach()) - f_ref) < 1e-4
    assert metrics.rel_l2(ang.grad.numpy(), g_ref) < GTOL


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp16"])
def test_gradient_on_a_split_precision_grid(precision):
    """A grid built for split-precision amplitudes runs its adjoint in complex64 (the
    gradient's products are complex64 whatever the grid's precision): same 1e-3 bound."""
    _need_gpu()
    _say("grad on a", precision, "grid")
    c = R.grid_rqc(4, 4, 12, 616, two_qubit="fsim", jitter_sd=0.02, jitter_seed=61)
    bits = R.bitstrings(16, 20, 617)
    res = build_grid(c, precision=precision).contract_grad(bits)
    f_ref, g_ref = E1.linear_xeb_grad(c, bits)
    assert metrics.rel_l2(res["grad_params"][0][_fsim_rows(c)], g_ref) < GTOL
    assert abs(res["loss"][0] - f_ref) < 1e-4 * max(1.0, abs(f_ref))


def test_autotuned_gradient_matches_shape_rule_gradient():
    """An autotuned grid times every fitting kernel of each forward and backward product (the
    MFMA rows and reduction kernels, split-K chunks included) and keeps the fastest: its
    gradients match the shape rules' within FP32 rounding, and the state-vector adjoint.  Both
    grids read some intermediates in place (forward, and transposed in the backward pass)."""
    _need_gpu()
    _say("autotuned gradient, 5x4 and 6x6 fSim")
    c1 = R.grid_rqc(5, 4, 12, 910, two_qubit="fsim", jitter_sd=0.02, jitter_seed=11)
    c2 = R.grid_rqc(6, 6, 12, 911, two_qubit="fsim", jitter_sd=0.02, jitter_seed=12)
    bits = [R.bitstrings(20, 64, 912), R.bitstrings(36, 64, 913)]
    tuned = build_grid([c1, c2], autotune=True)
    plain = build_grid([c1, c2])
    r_t = [tuned.contract_grad(bits) for _ in range(2)]  # the first call tunes
    plain.set_profiling(True)
    r_p = plain.contract_grad(bits)
    prof = plain.profile_read()
    # products that read their intermediate x in place, forward and (as X^T) backward
    assert prof["gemm_rows_mfma_gather_nn"]["launches"] > 0, prof.keys()
    assert prof["gemm_rows_mfma_gather_tn"]["launches"] > 0, prof.keys()
    for r in r_t:
        for ci, c in enumerate((c1, c2)):
            f = _fsim_rows(c)
            err = metrics.rel_l2(r["grad_params"][ci][f], r_p["grad_params"][ci][f])
            _say("  circuit", ci, "tuned vs shape rules", err)
            assert err < 1e-5
            assert abs(r["loss"][ci] - r_p["loss"][ci]) < 1e-5 * max(1.0, abs(r_p["loss"][ci]))
    f_ref, g_ref = E1.linear_xeb_grad(c1, bits[0])
    assert metrics.rel_l2(r_t[1]["grad_params"][0][_fsim_rows(c1)], g_ref) < GTOL
    assert abs(r_t[1]["loss"][0] - f_ref) < 1e-4 * max(1.0, abs(f_ref))
    tuned.close()
    plain.close()


@pytest.mark.parametrize("precision", ["c64", "split_bf16", "split_fp16"])
def test_update_gates_matches_a_fresh_grid(precision):
    """qflex_update_gates: the same fSim circuit with other angles, collapsed again in place,
    gives the amplitudes a grid built for it gives, bit for bit (same plan, same kernels); a
    circuit of another structure is rejected and leaves the grid as it was."""
    import torch

    from paper_1811_09599_amd import _ffi as F
    from paper_1811_09599_amd.qflex import with_fsim_angles

    _need_gpu()
    _say("update gates,", precision)
    c = R.grid_rqc(4, 4, 12, 4343, two_qubit="fsim", jitter_sd=0.02, jitter_seed=43)
    op = [15, 14]
    bits = R.bitstrings(16, 8, 44, op)
    rng = np.random.default_rng(45)
    c2 = with_fsim_angles(c, R.fsim_params(c) + rng.normal(0, 0.3, R.fsim_params(c).shape))
    g = build_grid(c, plan="quadrant", open_qubits=op, precision=precision)
    before = g.contract_amplitudes(bits, fidelity=0.5, seed=3)
    g.update_gates(c2)
    got = g.contract_amplitudes(bits, fidelity=0.5, seed=3)
    fresh = build_grid(c2, plan="quadrant", open_qubits=op, precision=precision)
    want = fresh.contract_amplitudes(bits, fidelity=0.5, seed=3)
    assert torch.equal(got, want)
    assert not torch.equal(got, before)
    cz = R.grid_rqc(4, 4, 12, 4343)  # CZ couplers: other kinds and ranks
    with pytest.raises(F.QflexError) as e:
        g.update_gates(cz)
    assert e.value.status == F.E_INVALID
    assert torch.equal(g.contract_amplitudes(bits, fidelity=0.5, seed=3), want)
    g.close()
    fresh.close()


def test_autograd_function_reuses_its_grid_across_angles():
    """Two forward passes at different angles share one grid (the second updates its gates);
    the backward pass of the first still differentiates at its own angles."""
    _need_gpu()
    import torch
    from paper_1811_09599_amd import Amplitudes
    from paper_1811_09599_amd.qflex import with_fsim_angles
    _say("autograd, shared grid")
    c = R.grid_rqc(3, 3, 12, 4242, two_qubit="fsim", jitter_sd=0.02, jitter_seed=42)
    bits = R.bitstrings(9, 16, 9)
    p0 = R.fsim_params(c)
    p1 = p0 + 0.1
    a0 = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    a1 = torch.tensor(p1, dtype=torch.float64, requires_grad=True)
    f0 = (2.0 ** 9) * torch.mean(Amplitudes.apply(a0, c, bits).abs() ** 2) - 1.0
    f1 = (2.0 ** 9) * torch.mean(Amplitudes.apply(a1, c, bits).abs() ** 2) - 1.0
    f0.backward()
    f1.backward()
    for a, p, f in ((a0, p0, f0), (a1, p1, f1)):
        f_ref, g_ref = E1.linear_xeb_grad(with_fsim_angles(c, p), bits)
        assert abs(float(f.detach()) - f_ref) < 1e-4
        assert metrics.rel_l2(a.grad.numpy(), g_ref) < GTOL


def _closed_expansion(bits, cot, op):
    """The open-batch amplitudes psi[b, i] as closed bit-strings: row b with the open qubits
    set to the big-endian digits of i, and the conjugated cotangent flattened the same way."""
    rows = []
    for b in range(len(bits)):
        for i in range(1 << len(op)):
            r = bits[b].copy()
            for j, q in enumerate(op):
                r[q] = (i >> (len(op) - 1 - j)) & 1
            rows.append(r)
    return np.array(rows, dtype=np.uint8), np.conj(cot).reshape(-1)


def test_degenerate_one_and_two_qubit_grid_gradients():
    """The adjoint on the smallest grids: one qubit (the result is the qubit tensor itself, its
    cotangent routed straight back into the gates) and two qubits in a row or a column (one
    product between two qubit tensors), closed and with open qubits, under a given cotangent:
    every gate's entry gradient and every fSim angle gradient against the state-vector
    adjoint."""
    _need_gpu()
    for rows, cols in ((1, 1), (1, 2), (2, 1)):
        c = R.grid_rqc(rows, cols, 8, 170 + 10 * rows + cols, two_qubit="fsim", jitter_sd=0.05,
                       jitter_seed=4)
        n = c["n_qubits"]
        for op in [[], [n - 1]] + ([list(range(n))] if n > 1 else []):
            _say("grad", rows, cols, "open", op)
            bits = R.bitstrings(n, 5, 40 + len(op), op)
            rng = np.random.default_rng(2 + len(op))
            cot = (rng.standard_normal((5, 1 << len(op)))
                   + 1j * rng.standard_normal((5, 1 << len(op))))
            g = build_grid(c, open_qubits=op)
            res = g.contract_grad(bits, cotangent=cot)
            g.close()
            full, w = _closed_expansion(bits, cot, op)
            amp = E1.amplitudes(c, full).reshape(5, 1 << len(op))
            assert metrics.amp_errors(res["amps"], amp, n)["max"] < 1e-5
            dgate = E1.vjp_gates(c, full, w)
            for i, gt in enumerate(c["gates"]):
                if gt["kind"] != "cz":
                    assert metrics.rel_l2(np.conj(res["grad_gates"][0][i]), dgate[i]) < GTOL, i
            fs = _fsim_rows(c)
            if fs:
                dth, dph, _ = E1.vjp_params(c, full, w)
                ref = np.stack([dth.real, dph.real], axis=1)
                assert metrics.rel_l2(res["grad_params"][0][fs], ref) < GTOL
