"""GPU parity of the whole contraction path (qflex_build_grid + qflex_contract_amplitudes)
against the CPU oracle, to 1e-5 relative error on 2^(n/2)-scaled amplitudes."""
import numpy as np
import pytest

import rqc_inputs as R
from oracle import metrics
from oracle import slices as OS
from oracle import statevector as E1
from oracle import tn as E2
from paper_1811_09599_amd import _ffi as F
from paper_1811_09599_amd import build_grid

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


def test_cfg1_4x4_depth16_256_amplitudes_vs_state_vector():
    _need_gpu()
    _say("cfg1 4x4 1+16+1")
    c = R.grid_rqc(4, 4, 16, 1001)
    bits = R.bitstrings(16, 256, 1500)
    g = build_grid(c)
    a = g.contract_amplitudes(bits).cpu().numpy()[:, 0]
    _check(a, E1.amplitudes(c, bits), 16)
    st = g.last_stats()
    assert st["n_bitstrings"] == 256 and st["n_slices"] == 1 and st["flops"] > 0


@pytest.mark.parametrize("rows,cols,depth,kind", [(2, 2, 8, "cz"), (2, 3, 16, "cz"),
                                                  (3, 3, 24, "cz"), (4, 5, 16, "cz"),
                                                  (3, 4, 12, "fsim"), (4, 4, 12, "fsim"),
                                                  (1, 5, 16, "cz")])
def test_sweep_plan_vs_state_vector(rows, cols, depth, kind):
    _need_gpu()
    _say("sweep", rows, cols, depth, kind)
    n = rows * cols
    c = R.grid_rqc(rows, cols, depth, 77 + n, two_qubit=kind, jitter_sd=0.02)
    bits = R.bitstrings(n, 37, 5)
    a = build_grid(c).contract_amplitudes(bits).cpu().numpy()[:, 0]
    _check(a, E1.amplitudes(c, bits), n)


def test_open_qubit_batch_covers_every_bitstring_and_is_normalised():
    _need_gpu()
    _say("normalisation 4x4 depth 24, 64-amplitude batches")
    c = R.grid_rqc(4, 4, 24, 21)
    op = [10, 11, 14, 15, 9, 13]
    closed = [q for q in range(16) if q not in op]
    rows = np.zeros((1 << len(closed), 16), dtype=np.uint8)
    for i in range(1 << len(closed)):
        for t, q in enumerate(closed):
            rows[i, q] = (i >> t) & 1
    a = build_grid(c, open_qubits=op).contract_amplitudes(rows).cpu().numpy()
    assert a.shape == (1 << 10, 64)
    assert abs(np.sum(np.abs(a) ** 2) - 1.0) < 1e-5
    _check(a, E1.amplitudes(c, rows, op), 16)


@pytest.mark.parametrize("rows,cols,depth,kind", [(4, 4, 16, "cz"), (4, 5, 24, "cz"),
                                                  (5, 4, 8, "cz"), (4, 4, 12, "fsim"),
                                                  (3, 3, 16, "cz")])
def test_quadrant_plan_all_slices_vs_state_vector(rows, cols, depth, kind):
    _need_gpu()
    _say("quadrant", rows, cols, depth, kind)
    n = rows * cols
    c = R.grid_rqc(rows, cols, depth, 300 + n, two_qubit=kind, jitter_sd=0.02)
    op = [n - 1, n - 2, n - cols - 1]
    bits = R.bitstrings(n, 9, 8, op)
    g = build_grid(c, plan="quadrant", open_qubits=op)
    assert len(g.plan_cuts()) == 2
    a = g.contract_amplitudes(bits).cpu().numpy()
    _check(a, E1.amplitudes(c, bits, op), n)
    assert g.last_stats()["n_slices"] == g.num_slices()


def test_quadrant_single_slices_match_oracle_paths():
    _need_gpu()
    _say("per-slice parity 4x5 depth 16")
    c = R.grid_rqc(4, 5, 16, 41)
    op = [19, 18]
    bits = R.bitstrings(20, 5, 3, op)
    g = build_grid(c, plan="quadrant", open_qubits=op)
    cuts = g.plan_cuts()
    S = g.num_slices()
    net = E2.Network(c)
    for s in (0, 1, S // 2 + 3, S - 1):
        a = g.contract_amplitudes(bits, slice_ids=[s]).cpu().numpy()
        ref = net.amplitudes(bits, op, cuts=cuts, slice_ids=[s]).numpy()
        _check(a, ref, 20)


@pytest.mark.parametrize("mode", ["random", "block"])
def test_low_fidelity_subset_matches_oracle_subset(mode):
    _need_gpu()
    _say("fidelity 1/4 on 4x4 depth 24,", mode)
    c = R.grid_rqc(4, 4, 24, 55)
    bits = R.bitstrings(16, 6, 2)
    g = build_grid(c, plan="quadrant", slice_mode=mode)
    S = g.num_slices()
    f, seed = 0.25, 2700
    a = g.contract_amplitudes(bits, fidelity=f, seed=seed).cpu().numpy()[:, 0]
    ids = OS.select(S, f, seed) if mode == "random" else OS.select_block(S, f, seed)
    assert g.last_stats()["n_slices"] == len(ids)
    ref = E2.amplitudes(c, bits, cuts=g.plan_cuts(), slice_ids=ids)
    _check(a, ref, 16)


def test_bitstring_batching_does_not_change_results():
    _need_gpu()
    _say("batching")
    c = R.grid_rqc(4, 4, 16, 9)
    bits = R.bitstrings(16, 11, 4, [15])
    outs = []
    for B in (1, 3, 0):
        g = build_grid(c, plan="quadrant", open_qubits=[15], bitstring_batch=B)
        outs.append(g.contract_amplitudes(bits).cpu().numpy())
    assert np.allclose(outs[0], outs[1], rtol=0, atol=1e-12)
    assert np.allclose(outs[0], outs[2], rtol=0, atol=1e-12)
    g2 = build_grid(c, plan="quadrant", open_qubits=[15])
    r1 = g2.contract_amplitudes(bits).cpu().numpy()
    r2 = g2.contract_amplitudes(bits).cpu().numpy()
    assert np.array_equal(r1, r2)  # deterministic


def test_many_circuits_in_one_call_with_host_output():
    _need_gpu()
    _say("batch of uneven circuits")
    cs = R.fsim_batch(4, depth=12, sizes=(3, 4))
    bits = [R.bitstrings(c["n_qubits"], 5 + i, 40 + i) for i, c in enumerate(cs)]
    bits[2] = bits[2][:0]  # a circuit with no bit-strings
    g = build_grid(cs)
    a = g.contract_amplitudes(bits, device=False)
    off = 0
    for c, b in zip(cs, bits):
        ref = E1.amplitudes(c, b)
        _check(a[off:off + len(b), 0], ref, c["n_qubits"])
        off += len(b)
    assert off == a.shape[0]


def test_edge_cases():
    _need_gpu()
    _say("edge cases")
    one = {"n_qubits": 1, "xy": [[0, 0]], "depth": 1,
           "gates": [{"cycle": 0, "kind": "h", "qubits": [0]},
                     {"cycle": 1, "kind": "t", "qubits": [0]},
                     {"cycle": 2, "kind": "h", "qubits": [0]}]}
    b = np.array([[0], [1]], dtype=np.uint8)
    a = build_grid(one).contract_amplitudes(b).cpu().numpy()[:, 0]
    assert np.allclose(a, E1.amplitudes(one, b), atol=1e-7)
    a = build_grid(one, open_qubits=[0]).contract_amplitudes(b[:1]).cpu().numpy()
    assert np.allclose(a[0], E1.amplitudes(one, b[:1], [0])[0], atol=1e-7)
    # depth 1+0+1 is the identity: psi = delta_{x,0}
    c0 = R.grid_rqc(3, 3, 0, 1)
    bits = R.bitstrings(9, 8, 1)
    bits[0] = 0
    a = build_grid(c0).contract_amplitudes(bits).cpu().numpy()[:, 0]
    want = np.array([1.0 if not x.any() else 0.0 for x in bits])
    assert np.allclose(a, want, atol=1e-6)
    # invalid calls are rejected without launching
    g = build_grid(R.grid_rqc(3, 3, 8, 2), plan="quadrant")
    bad = np.full((2, 9), 2, dtype=np.uint8)
    with pytest.raises(F.QflexError) as e:
        g.contract_amplitudes(bad)
    assert e.value.status == F.E_INVALID
    with pytest.raises(F.QflexError) as e:
        g.contract_amplitudes(np.zeros((1, 9), np.uint8), slice_ids=[g.num_slices()])
    assert e.value.status == F.E_INVALID
    with pytest.raises(F.QflexError) as e:
        g.contract_amplitudes(np.zeros((1, 9), np.uint8), fidelity=0.3)
    assert e.value.status == F.E_PLAN
    # empty call
    assert g.contract_amplitudes(np.zeros((0, 9), np.uint8)).shape == (0, 1)


def test_cfg2_7x7_depth32_sampled_slices_vs_oracle():
    """Full-size 7x7 (1+32+1) quadrant plan with a 64-amplitude open batch: one bit-string,
    two slices, compared slice by slice with the FP64 contraction of the same paths."""
    _need_gpu()
    _say("7x7 1+32+1 per-slice parity")
    c = R.grid_rqc(7, 7, 32, 2001)
    op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    bits = R.bitstrings(49, 1, 2500, op)
    g = build_grid(c, open_qubits=op)
    cuts = g.plan_cuts()
    assert g.num_slices() == 256
    ids = [37, 200]
    a = g.contract_amplitudes(bits, slice_ids=ids).cpu().numpy()
    order = E2.quadrant_order(7, 7)
    ref = E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=ids, order=order)
    _say("oracle done")
    _check(a, ref, 49)


def test_bench_launch_configuration_7x7():
    """The headline's own configuration: the bench circuit and its first step (8 bit-strings
    in one call, all 256 slices, autotuned split-bf16 products).  At that size the FP64 oracle
    affords single slices only, so: (1) two slices of the 8-bit-string call match the oracle;
    (2) the all-slice call equals the sum of its 256 single-slice calls (a property at any
    size: the amplitude is the sum of its paths)."""
    _need_gpu()
    _say("bench configuration: 7x7 1+32+1, 8 bit-strings, all slices, split-bf16, autotune")
    c = R.grid_rqc(7, 7, 32, 2000)
    op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    bits = R.bitstrings(49, 1024, 2500, op)[:8]
    g = build_grid(c, open_qubits=op, precision="split_bf16", autotune=True)
    full = g.contract_amplitudes(bits).cpu().numpy()  # tunes on this call
    full = g.contract_amplitudes(bits).cpu().numpy()
    cuts = g.plan_cuts()
    order = E2.quadrant_order(7, 7)
    for sid in (5, 250):
        one = g.contract_amplitudes(bits, slice_ids=[sid]).cpu().numpy()
        ref = E2.amplitudes(c, bits[:1], op, cuts=cuts, slice_ids=[sid], order=order)
        e = _check(one[:1], ref, 49, SPLIT_TOL["split_bf16"])
        _say("  slice", sid, e)
    total = np.zeros_like(full)
    for sid in range(g.num_slices()):
        total += g.contract_amplitudes(bits, slice_ids=[sid]).cpu().numpy()
    e = _check(full, total, 49, SPLIT_TOL["split_bf16"])
    _say("  all slices vs sum of single slices", e)
    g.close()


@pytest.mark.parametrize("prec", ["c64", "split_bf16", "split_fp16"])
def test_fsim_7x7_depth16_sampled_slices_vs_oracle(prec):
    """fSim couplers (rank-4 bonds, 2 bond bits per gate): a 1+16+1 fSim circuit has the bond
    dimensions of a 1+32+1 CZ circuit (16 per link), and its 7x7 contraction runs the same
    quadrant plan, checked slice by slice against the FP64 contraction."""
    _need_gpu()
    _say(prec, "7x7 fSim 1+16+1 per-slice parity")
    c = R.grid_rqc(7, 7, 16, 2002, two_qubit="fsim", jitter_sd=0.02, jitter_seed=3)
    op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    bits = R.bitstrings(49, 1, 2501, op)
    g = build_grid(c, open_qubits=op, precision=prec)
    assert g.num_slices() == 256
    ids = [11, 190]
    g.set_profiling(True)
    a = g.contract_amplitudes(bits, slice_ids=ids).cpu().numpy()
    prof = g.profile_read()
    ref = E2.amplitudes(c, bits, op, cuts=g.plan_cuts(), slice_ids=ids,
                        order=E2.quadrant_order(7, 7))
    _say("oracle done")
    e = _check(a, ref, 49, SPLIT_TOL.get(prec, 1e-5))
    _say("  error", e)
    # the plan's two (2^16 or 2^12, 256, 16) steps read their intermediate x in its storage
    # order (no permutation pass), and so do A.B and AB.D their column operands: this parity
    # check covers those paths
    assert prof["gemm_rows_mfma_gather_nn"]["launches"] == 2 * len(ids), prof.keys()
    if prec != "c64":
        fmt = prec.split("_")[1]
        assert prof["gemm_split3m_%s_gatherb_256x128" % fmt]["launches"] >= len(ids), prof.keys()


# ------------------------------------------------------------------- cut sweeps
@pytest.mark.parametrize("layout", ["grid4x5", "diamond15"])
def test_cut_sweep_all_slices_vs_state_vector(layout):
    """Links cut until every intermediate fits a small cap: the sum over all slices is the
    amplitude (slicing is exact), on a grid and on a corner of the diamond lattice."""
    _need_gpu()
    _say("cut sweep", layout)
    if layout == "grid4x5":
        c, cap, op = R.grid_rqc(4, 5, 16, 4242), 1 << 8, [19, 18]
    else:
        c, cap, op = R.rqc([p for p in R.diamond_layout() if p[0] <= 3], 16, 77), 1 << 7, [0, 1]
    n = c["n_qubits"]
    bits = R.bitstrings(n, 3, 91, op)
    g = build_grid(c, plan="cut_sweep", max_tensor_elems=cap, open_qubits=op)
    assert g.num_slices() >= 64
    a = g.contract_amplitudes(bits).cpu().numpy()
    e = _check(a, E1.amplitudes(c, bits, op), n)
    _say("  error", e, "slices", g.num_slices())


def test_cut_sweep_single_slices_match_oracle_paths():
    _need_gpu()
    c = R.grid_rqc(4, 5, 16, 4343)
    op = [19, 18]
    bits = R.bitstrings(20, 2, 92, op)
    g = build_grid(c, plan="cut_sweep", max_tensor_elems=1 << 8, open_qubits=op)
    S = g.num_slices()
    ids = [0, 17, S - 1]
    a = g.contract_amplitudes(bits, slice_ids=ids).cpu().numpy()
    ref = E2.amplitudes(c, bits, op, cuts=g.plan_cuts(), slice_ids=ids)
    _check(a, ref, 20)


# ------------------------------------------------------------------- split precisions
# Stated bounds: split-bf16 keeps ~16 of an operand's 24 bits (bf16x3 products, FP32
# accumulation); split-fp16 keeps ~22 (inside its scale window), so its bound is 4x the
# complex64 bound.
SPLIT_TOL = {"split_bf16": 2e-4, "split_fp16": 4 * TOL}


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_quadrant_5x4_depth32_vs_state_vector(prec):
    _need_gpu()
    _say(prec, "5x4 1+32+1 quadrant")
    c = R.grid_rqc(5, 4, 32, 5432)
    op = [19, 18, 15]
    bits = R.bitstrings(20, 6, 7, op)
    g = build_grid(c, plan="quadrant", open_qubits=op, precision=prec)
    g.set_profiling(True)
    a = g.contract_amplitudes(bits).cpu().numpy()
    prof = g.profile_read()
    assert any(k.startswith("gemm_" + prec) for k in prof), prof
    e = _check(a, E1.amplitudes(c, bits, op), 20, SPLIT_TOL[prec])
    _say("  split error", e)
    ref_c64 = build_grid(c, plan="quadrant", open_qubits=op).contract_amplitudes(bits)
    _say("  c64 error", metrics.amp_errors(ref_c64.cpu().numpy(), E1.amplitudes(c, bits, op), 20))


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_7x7_depth32_sampled_slices_vs_oracle(prec):
    _need_gpu()
    _say(prec, "7x7 1+32+1 per-slice parity")
    c = R.grid_rqc(7, 7, 32, 2001)
    op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    bits = R.bitstrings(49, 1, 2500, op)
    g = build_grid(c, open_qubits=op, precision=prec)
    ids = [37, 200]
    a = g.contract_amplitudes(bits, slice_ids=ids).cpu().numpy()
    ref = E2.amplitudes(c, bits, op, cuts=g.plan_cuts(), slice_ids=ids,
                        order=E2.quadrant_order(7, 7))
    e = _check(a, ref, 49, SPLIT_TOL[prec])
    _say("  split error", e)


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_cut_sweep_slices_match_oracle_paths(prec):
    """Split products on a cut-sweep layout (4x5, depth 1+32+1, four cut links under a 2^16
    cap): gathered and pre-split operands in shapes the quadrant plans do not produce, checked
    slice by slice against the FP64 contraction of the same paths."""
    _need_gpu()
    _say(prec, "cut sweep 4x5 1+32+1 per-slice parity")
    c = R.grid_rqc(4, 5, 32, 4242)
    op = [19, 18]
    bits = R.bitstrings(20, 3, 93, op)
    g = build_grid(c, plan="cut_sweep", max_tensor_elems=1 << 16, open_qubits=op,
                   precision=prec, autotune=True)
    S = g.num_slices()
    ids = [0, 4097, S // 2 + 3, S - 1]
    a = g.contract_amplitudes(bits, slice_ids=ids).cpu().numpy()
    ref = E2.amplitudes(c, bits, op, cuts=g.plan_cuts(), slice_ids=ids)
    e = _check(a, ref, 20, SPLIT_TOL[prec])
    _say("  error", e)


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_many_circuits_in_one_call(prec):
    """Uneven circuits in one call (one with no bit-strings) in split precision, against the
    state vector."""
    _need_gpu()
    _say(prec, "batch of uneven circuits")
    cs = [R.grid_rqc(4, 4, 24, 60), R.grid_rqc(3, 5, 24, 61), R.grid_rqc(4, 5, 24, 62)]
    bits = [R.bitstrings(c["n_qubits"], 4 + i, 50 + i) for i, c in enumerate(cs)]
    bits[1] = bits[1][:0]
    g = build_grid(cs, precision=prec)
    a = g.contract_amplitudes(bits, device=False)
    off = 0
    for c, b in zip(cs, bits):
        _check(a[off:off + len(b), 0], E1.amplitudes(c, b), c["n_qubits"], SPLIT_TOL[prec])
        off += len(b)
    assert off == a.shape[0]


@pytest.mark.parametrize("mode", ["random", "block"])
def test_split_low_fidelity_subset_matches_oracle_subset(mode):
    """A fidelity-1/4 slice subset (random or block) in split-bf16 on the 5x4 depth-32 quadrant
    plan: intermediates reused across the subset's slices go through the split cache."""
    _need_gpu()
    _say("split-bf16 fidelity 1/4 on 5x4 depth 32,", mode)
    c = R.grid_rqc(5, 4, 32, 5433)
    op = [19, 18]
    bits = R.bitstrings(20, 4, 3, op)
    g = build_grid(c, plan="quadrant", open_qubits=op, precision="split_bf16", slice_mode=mode)
    S = g.num_slices()
    f, seed = 0.25, 2701
    a = g.contract_amplitudes(bits, fidelity=f, seed=seed).cpu().numpy()
    ids = OS.select(S, f, seed) if mode == "random" else OS.select_block(S, f, seed)
    assert g.last_stats()["n_slices"] == len(ids)
    ref = E2.amplitudes(c, bits, op, cuts=g.plan_cuts(), slice_ids=ids)
    e = _check(a, ref, 20, SPLIT_TOL["split_bf16"])
    _say("  error", e)


@pytest.mark.parametrize("prec", ["c64", "split_bf16"])
def test_degenerate_one_and_two_qubit_grids(prec):
    """The smallest grids: one qubit (no product at all: the amplitude is the collapsed qubit
    tensor itself) and two qubits in a row or a column (one product), with every qubit closed
    or open, against the state vector."""
    _need_gpu()
    _say("1x1, 1x2, 2x1 grids,", prec)
    for rows, cols in ((1, 1), (1, 2), (2, 1)):
        c = R.grid_rqc(rows, cols, 4, 70 + 10 * rows + cols)
        n = c["n_qubits"]
        for op in ([], [0], list(range(n))):
            bits = R.bitstrings(n, 3, 90 + len(op), op)
            g = build_grid(c, open_qubits=op, precision=prec)
            a = g.contract_amplitudes(bits).cpu().numpy()
            g.close()
            _check(a, E1.amplitudes(c, bits, op), n, SPLIT_TOL.get(prec, TOL))
