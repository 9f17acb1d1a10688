"""Pins of the CPU oracle against things other than itself: textbook identities, closed
forms, special cases, the other engine, finite differences and the paper's own numbers."""
import itertools
import math
import os

import numpy as np
import pytest

import rqc_inputs as R
from oracle import gates as G
from oracle import metrics, slices
from oracle import statevector as E1
from oracle import tn as E2

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- gates
def test_one_qubit_gates_are_textbook_roots():
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    S = np.diag([1, 1j])
    assert np.allclose(G.X12 @ G.X12, X)
    assert np.allclose(G.Y12 @ G.Y12, Y)
    assert np.allclose(G.T @ G.T, S)
    assert np.allclose(np.linalg.matrix_power(G.T, 8), np.eye(2))
    assert np.allclose(G.H @ G.H, np.eye(2))
    assert np.allclose(G.H @ np.diag([1, -1]) @ G.H, X)
    for m in (G.H, G.X12, G.Y12, G.T, G.CZ, G.fsim(0.3, 1.1)):
        assert np.allclose(m.conj().T @ m, np.eye(len(m)))


def test_fsim_special_cases_match_paper_iswap_and_cz():
    rows = [l.split() for l in open(os.path.join(GOLD, "iswap_methods_a.txt"))
            if l.strip() and not l.startswith("#")]
    iswap = np.array([[float(r[2 * j]) + 1j * float(r[2 * j + 1]) for j in range(4)]
                      for r in rows])
    assert np.allclose(G.fsim(-np.pi / 2, 0.0), iswap)
    assert np.allclose(G.fsim(0.0, np.pi), G.CZ)
    assert np.allclose(G.fsim(0.0, 0.0), np.eye(4))


def test_fsim_derivatives_match_finite_differences():
    t, p, h = 0.7, -0.4, 1e-6
    assert np.allclose((G.fsim(t + h, p) - G.fsim(t - h, p)) / (2 * h), G.dfsim_dtheta(t, p),
                       atol=1e-9)
    assert np.allclose((G.fsim(t, p + h) - G.fsim(t, p - h)) / (2 * h), G.dfsim_dphi(t, p),
                       atol=1e-9)


def test_bond_decomposition_reassembles_gate():
    import torch
    for mat, rank in ((G.CZ, 2), (G.fsim(0.0, 0.4), 2), (G.fsim(1.3, 0.4), 4),
                      (G.fsim(-np.pi / 2, 0), 4)):
        pieces = E2.split_two_qubit(torch.as_tensor(mat))
        assert len(pieces) == rank
        acc = sum(np.kron(a.numpy(), b.numpy()) for a, b in pieces)
        assert np.allclose(acc, mat, atol=0, rtol=0)


# ----------------------------------------------------------------------------- generator
def test_generator_follows_rqc_rules():
    c = R.grid_rqc(5, 6, 24, 3)
    n = c["n_qubits"]
    by_cycle = {}
    for g in c["gates"]:
        by_cycle.setdefault(g["cycle"], []).append(g)
    # rules (1) and (5): H first and last on every qubit
    assert sorted(g["qubits"][0] for g in by_cycle[0]) == list(range(n))
    assert sorted(g["qubits"][0] for g in by_cycle[25]) == list(range(n))
    prev = {q: "h" for q in range(n)}
    for cyc in range(1, 25):
        seen = {}
        for g in by_cycle.get(cyc, []):
            for q in g["qubits"]:
                assert q not in seen  # every layer is a matching on disjoint qubits
                seen[q] = g["kind"]
        for q in range(n):
            k = seen.get(q, "")
            if k == "t":
                assert prev[q] in ("x12", "y12", "h")  # rule (4); never T right after CZ
            if k in ("x12", "y12"):
                assert prev[q] == "cz"  # rule (3)
            if prev[q] == "cz" and k != "cz":
                assert k in ("x12", "y12")
            prev[q] = k
    # each link carries exactly one CZ per eight cycles (Methods B)
    for start in (1, 9, 17):
        cnt = {}
        for cyc in range(start, start + 8):
            for g in by_cycle.get(cyc, []):
                if g["kind"] == "cz":
                    cnt[tuple(g["qubits"])] = cnt.get(tuple(g["qubits"]), 0) + 1
        assert set(cnt) == set(R.couplers(c["xy"])) and set(cnt.values()) == {1}
    # no two horizontal / vertical layers in a row
    for a, b in zip(R.LAYER_ORDER, R.LAYER_ORDER[1:] + R.LAYER_ORDER[:1]):
        assert a[0] != b[0]


def test_diamond_layout_matches_paper_geometry():
    xy = R.diamond_layout()
    assert len(xy) == 70  # Bristlecone-72 minus its two single-neighbour corners
    cps = R.couplers(xy)
    assert len(cps) == 119
    xs = [p[0] for p in xy]
    ys = [p[1] for p in xy]
    assert (max(xs) - min(xs) + 1, max(ys) - min(ys) + 1) in ((10, 11), (11, 10))


# ----------------------------------------------------------------------------- E1 pins
def _all_bits(n):
    return np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.uint8)


def test_e1_norm_and_trivial_depth():
    c = R.grid_rqc(3, 3, 16, 11)
    psi = E1.state(c)
    assert abs(np.sum(np.abs(psi) ** 2) - 1) < 1e-12
    c0 = R.grid_rqc(3, 3, 0, 1)  # depth 1+0+1: H then H
    psi0 = E1.state(c0).ravel()
    want = np.zeros_like(psi0)
    want[0] = 1
    assert np.allclose(psi0, want, atol=1e-14)


def _cz_closed_form(c, x):
    """CZ-only circuit between H layers: psi(x) = 2^-n sum_y (-1)^(x.y + sum_CZ y_a y_b)."""
    n = c["n_qubits"]
    ys = _all_bits(n).astype(np.int64)
    ph = ys @ np.asarray(x, dtype=np.int64)
    for g in c["gates"]:
        if g["kind"] == "cz":
            a, b = g["qubits"]
            ph = ph + ys[:, a] * ys[:, b]
    return np.sum((-1.0) ** (ph % 2)) / 2 ** n


@pytest.mark.parametrize("engine", ["E1", "E2"])
def test_cz_only_circuit_matches_walsh_hadamard_closed_form(engine):
    c = R.without_kinds(R.grid_rqc(3, 4, 16, 5), ("x12", "y12", "t"))
    bits = R.bitstrings(12, 12, 9)
    got = E1.amplitudes(c, bits) if engine == "E1" else E2.amplitudes(c, bits)
    want = np.array([_cz_closed_form(c, x) for x in bits])
    assert np.allclose(got, want, atol=1e-13)


@pytest.mark.parametrize("engine", ["E1", "E2"])
def test_clifford_variant_has_flat_nonzero_probabilities(engine):
    c = R.without_kinds(R.grid_rqc(3, 3, 16, 2), ("t",))
    bits = _all_bits(9)
    p = np.abs(E1.amplitudes(c, bits) if engine == "E1" else E2.amplitudes(c, bits)) ** 2
    nz = p[p > 1e-12]
    r = -math.log2(nz[0])
    assert abs(r - round(r)) < 1e-9 and np.allclose(nz, 2.0 ** -round(r))
    assert abs(nz.sum() - 1) < 1e-12 and (len(nz) & (len(nz) - 1)) == 0


@pytest.mark.parametrize("engine", ["E1", "E2"])
def test_identity_coupling_gives_product_state(engine):
    c = R.replace_two_qubit(R.grid_rqc(3, 3, 16, 4), "fsim", 0.0, 0.0)
    bits = R.bitstrings(9, 10, 1)
    got = E1.amplitudes(c, bits) if engine == "E1" else E2.amplitudes(c, bits)
    single = {q: np.array([1, 0], dtype=complex) for q in range(9)}
    for g in sorted(c["gates"], key=lambda g: g["cycle"]):
        if len(g["qubits"]) == 1:
            q = g["qubits"][0]
            single[q] = G.matrix(g) @ single[q]
    want = np.array([np.prod([single[q][x[q]] for q in range(9)]) for x in bits])
    assert np.allclose(got, want, atol=1e-13)


def test_porter_thomas_second_moment_at_depth_24():
    c = R.grid_rqc(4, 4, 24, 21)
    p = np.abs(E1.state(c).ravel()) ** 2
    n = 16
    assert abs(np.mean(2 ** n * p) - 1) < 1e-12
    assert abs(2 ** n * np.sum(p ** 2) - 2.0) < 0.1  # Porter-Thomas: E[(Np)^2] = 2


# ----------------------------------------------------------------------------- E1 == E2
@pytest.mark.parametrize("shape,depth,kind", [((2, 2), 8, "cz"), ((2, 3), 16, "cz"),
                                              ((3, 3), 16, "cz"), ((3, 4), 24, "cz"),
                                              ((4, 4), 16, "cz"), ((3, 3), 12, "fsim"),
                                              ((2, 4), 12, "fsim")])
def test_e1_equals_e2(shape, depth, kind):
    r, cc = shape
    c = R.grid_rqc(r, cc, depth, 31 + r * cc, two_qubit=kind, jitter_sd=0.02)
    bits = R.bitstrings(r * cc, 16, 5)
    a1 = E1.amplitudes(c, bits)
    a2 = E2.amplitudes(c, bits)
    assert metrics.amp_errors(a2, a1, r * cc)["max"] < 1e-11


def test_e1_equals_e2_with_open_qubits():
    c = R.grid_rqc(3, 3, 16, 8)
    op = [6, 7, 8, 3]
    bits = R.bitstrings(9, 6, 2, op)
    a1 = E1.amplitudes(c, bits, op)
    a2 = E2.amplitudes(c, bits, op)
    assert a1.shape == (6, 16) and np.allclose(a1, a2, atol=1e-14)


def test_diamond_subgraph_e1_equals_e2():
    # a small corner of the diamond layout exercises non-rectangular neighbourhoods
    xy = [p for p in R.diamond_layout() if p[0] <= 2]
    c = R.rqc(xy, 16, 3)
    n = len(xy)
    assert 6 <= n <= 14
    bits = R.bitstrings(n, 8, 3)
    assert np.allclose(E1.amplitudes(c, bits), E2.amplitudes(c, bits), atol=1e-13)


# ----------------------------------------------------------------------------- slicing
def _path_replacements(c, cut_links, values):
    """Gate replacements that pin one path: each gate on a cut link keeps only its bond term
    A_k (x) B_k, k = the link value's digit for that gate (earliest gate most significant)."""
    import torch
    rep = {}
    for link, v in zip(cut_links, values):
        idx = [i for i, g in enumerate(c["gates"]) if len(g["qubits"]) == 2
               and tuple(sorted(g["qubits"])) == tuple(sorted(link))]
        ranks = []
        terms = []
        for i in idx:
            g = c["gates"][i]
            assert g["qubits"][0] < g["qubits"][1]
            p = E2.split_two_qubit(torch.as_tensor(G.matrix(g)))
            ranks.append(len(p))
            terms.append([np.kron(a.numpy(), b.numpy()) for a, b in p])
        digits = []
        for r in reversed(ranks):
            digits.append(v % r)
            v //= r
        for i, t, k in zip(idx, terms, reversed(digits)):
            rep[i] = t[k]
    return rep


@pytest.mark.parametrize("kind", ["cz", "fsim"])
def test_e2_path_equals_state_vector_path(kind):
    c = R.grid_rqc(3, 3, 16 if kind == "cz" else 10, 12, two_qubit=kind, jitter_sd=0.02)
    cuts = [(2, 5), (6, 7)]
    dims = E2.Network(c).cut_dims(cuts)
    bits = R.bitstrings(9, 4, 4)
    for s in (0, 1, dims[1], dims[0] * dims[1] - 1, 5):
        vals = [s // dims[1], s % dims[1]]
        psi_p = E1.state(c, _path_replacements(c, cuts, vals))
        want = np.array([psi_p[tuple(x)] for x in bits])
        got = E2.amplitudes(c, bits, cuts=cuts, slice_ids=[s])
        assert np.allclose(got, want, atol=1e-14), s


def test_sum_of_paths_is_the_amplitude_and_order_invariant():
    c = R.grid_rqc(3, 4, 16, 13)
    bits = R.bitstrings(12, 5, 6)
    op = [8, 9]
    cuts = [(3, 7), (9, 10)]
    net = E2.Network(c)
    S = int(np.prod(net.cut_dims(cuts)))
    full = E1.amplitudes(c, bits, op)
    summed = E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=range(S))
    assert np.allclose(summed, full, atol=1e-13)
    other = [("region", [0, 1, 4, 5]), ("region", [2, 3, 6, 7]), ("sweep", [8, 9, 10, 11])]
    a = E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=[3, 7], order=other)
    b = E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=[3, 7])
    assert np.allclose(a, b, atol=1e-14)


def test_low_fidelity_fraction_of_paths_eq1():
    """Eq. (1): summing a fraction f of the paths gives norm ~ f and fidelity ~ f."""
    c = R.grid_rqc(3, 4, 24, 7)
    cuts = [(3, 7), (9, 10)]
    dims = E2.Network(c).cut_dims(cuts)
    S = dims[0] * dims[1]
    paths = [E1.state(c, _path_replacements(c, cuts, [s // dims[1], s % dims[1]])).ravel()
             for s in range(S)]
    psi = np.sum(paths, axis=0)
    for f, seed in ((0.25, 1), (1 / 16, 2)):
        sel = slices.select(S, f, seed)
        pt = np.sum([paths[s] for s in sel], axis=0)
        nrm = np.vdot(pt, pt).real
        fid = abs(np.vdot(psi, pt)) ** 2 / nrm
        assert 0.8 * f < nrm < 1.25 * f
        assert 0.7 * f < fid < 1.4 * f


# ----------------------------------------------------------------------------- slices RNG
def test_splitmix64_reference_outputs():
    want = [int(l) for l in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    g = slices.SplitMix64(1234567)
    assert [g.next() for _ in range(5)] == want


def test_block_slice_selection_uses_the_first_splitmix64_output():
    """Block mode: the block index is the first SplitMix64 output (pinned by the published
    reference values) modulo the number of blocks; the block is k aligned consecutive ids."""
    first = int([l for l in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
                 if l.strip() and not l.startswith("#")][0])
    for total, f in ((1024, 1 / 64), (256, 1 / 4), (96, 0.25), (8, 1.0)):
        k = int(round(total * f))
        j = first % (total // k)
        assert slices.select_block(total, f, 1234567) == list(range(j * k, (j + 1) * k))
    with pytest.raises(ValueError):
        slices.select_block(12, 5 / 12, 1)


def test_slice_selection_properties():
    s = slices.select(1024, 1 / 64, 700)
    assert len(s) == 16 and s == sorted(s) and len(set(s)) == 16 and 0 <= s[0] and s[-1] < 1024
    assert slices.select(8, 1.0, 3) == list(range(8))
    with pytest.raises(ValueError):
        slices.select(10, 0.25, 1)
    with pytest.raises(ValueError):
        slices.select(10, 0.0, 1)


# ----------------------------------------------------------------------------- gradients
def test_e1_gradient_matches_central_differences():
    c = R.grid_rqc(2, 3, 12, 3, two_qubit="fsim", jitter_sd=0.02)
    bits = R.bitstrings(6, 10, 3)
    f, g = E1.linear_xeb_grad(c, bits)
    p0 = R.fsim_params(c)
    h = 1e-6
    fd = np.zeros_like(p0)
    for i in range(p0.shape[0]):
        for j in range(2):
            pp, pm = p0.copy(), p0.copy()
            pp[i, j] += h
            pm[i, j] -= h
            fd[i, j] = (E1.linear_xeb(R.with_fsim_params(c, pp), bits)
                        - E1.linear_xeb(R.with_fsim_params(c, pm), bits)) / (2 * h)
    assert metrics.rel_l2(g, fd) < 1e-6
    assert abs(f - E1.linear_xeb(c, bits)) < 1e-12


def test_gradient_euler_identity():
    """psi is linear in each gate's entries: sum_e dpsi/dG[e] * G[e] = psi for every gate."""
    c = R.grid_rqc(2, 3, 12, 5, two_qubit="fsim", jitter_sd=0.02)
    bits = R.bitstrings(6, 1, 8)
    dg = E1.vjp_gates(c, bits, np.ones(1))
    psi = E1.amplitudes(c, bits)[0]
    for i, g in enumerate(c["gates"]):
        assert abs(np.sum(dg[i] * G.matrix(g)) - psi) < 1e-14


def test_e3_autograd_equals_e1_adjoint():
    c = R.grid_rqc(3, 3, 12, 9, two_qubit="fsim", jitter_sd=0.02)
    bits = R.bitstrings(9, 12, 4)
    f1, g1 = E1.linear_xeb_grad(c, bits)
    f3, g3 = E2.linear_xeb_grad(c, bits)
    assert abs(f1 - f3) < 1e-12 and metrics.rel_l2(g3, g1) < 1e-10
    cot = np.exp(1j * np.arange(12)) * (1 + 0.1 * np.arange(12))
    dth, dph, _ = E1.vjp_params(c, bits, np.conj(cot))
    g_e1 = np.stack([dth.real, dph.real], axis=1)
    assert metrics.rel_l2(E2.amplitude_gate_grads(c, bits, cot), g_e1) < 1e-10


# ----------------------------------------------------------------------------- paper numbers
def test_frugal_acceptance_numbers_of_methods_c2():
    rows = [l.split() for l in open(os.path.join(GOLD, "frugal_acceptance_c2.txt"))
            if l.strip() and not l.startswith("#")]
    for m, nc, acc, batches in rows:
        p = 1 - (1 - 1 / int(m)) ** int(nc)
        assert abs(p - float(acc)) < 6e-5
        assert abs(1e6 / p - float(batches)) / float(batches) < 2e-3


def test_permutation_worked_example_moves_compose():
    steps = [l.split() for l in open(os.path.join(GOLD, "permutation_b2.txt"))
             if l.strip() and not l.startswith("#")]
    prev = steps[0][1].replace("|", "")
    for name, after in steps[1:-1]:
        cur = after.replace("|", "")
        assert sorted(cur) == sorted(prev)
        gamma = int(name[1:])
        if name[0] == "L":  # left move: the rightmost gamma indexes stay in place
            assert cur[-gamma:] == prev[-gamma:]
        else:  # right move: the leftmost indexes stay in place
            assert cur[:-gamma] == prev[:-gamma]
        prev = cur
    assert prev == steps[-1][1]


def test_e3_sliced_gradient_sums_to_full():
    """Gradients of a partial sum of paths add up to the full gradient over all paths."""
    c = R.grid_rqc(3, 3, 12, 19, two_qubit="fsim", jitter_sd=0.02)
    bits = R.bitstrings(9, 4, 2, [8])
    cot = np.exp(1j * np.arange(8)).reshape(4, 2)
    cuts = [(5, 8)]
    S = E2.num_slices(c, cuts)
    parts = [E2.amplitude_gate_grads(c, bits, cot, [8], cuts, [s]) for s in range(S)]
    full = E2.amplitude_gate_grads(c, bits, cot, [8])
    assert np.allclose(np.sum(parts, axis=0), full, atol=1e-12)


def test_identity_coupled_path_closed_form_matches_state_vector_paths():
    c = R.replace_two_qubit(R.grid_rqc(3, 3, 16, 23), "fsim", 0.0, 0.0)
    cuts = [(2, 5), (6, 7)]
    op = [8, 7]
    bits = R.bitstrings(9, 3, 4, op)
    dims = E2.Network(c).cut_dims(cuts)
    for s in (0, 3, dims[0] * dims[1] - 1, 6):
        vals = [s // dims[1], s % dims[1]]
        psi_p = E1.state(c, _path_replacements(c, cuts, vals))
        want = np.array([[psi_p[tuple(np.where(np.arange(9) == 8, (j >> 1) & 1,
                                                np.where(np.arange(9) == 7, j & 1, x)))]
                          for j in range(4)] for x in bits])
        got = E1.identity_coupled_path_amplitudes(c, bits, op, cuts, s)
        assert np.allclose(got, want, atol=1e-14), s
        assert np.allclose(got, E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=[s]), atol=1e-14)
