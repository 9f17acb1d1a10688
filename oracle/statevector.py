"""E1: FP64 state-vector simulator and its adjoint gradient.  TEST INFRASTRUCTURE (see
``oracle/__init__.py``).

What it computes is the plain definition the contraction reaches by other means: the
amplitude psi(x) = <x| U |0^n> of the circuit U (paper, Methods B: a circuit with fixed
input and output configurations closes into a tensor network whose value is this
amplitude).  The state is a numpy array of shape (2,)*n whose axis q is qubit q, so
``psi[x_0, ..., x_{n-1}]`` is the amplitude of bit-string x.  Gates are applied in cycle
order; gates inside one cycle act on disjoint qubits and commute.
"""
from __future__ import annotations

import numpy as np

from . import gates as G


def _ordered(circ):
    return sorted(range(len(circ["gates"])), key=lambda i: circ["gates"][i]["cycle"])


def _apply(psi: np.ndarray, mat: np.ndarray, qubits) -> np.ndarray:
    """Return mat applied to the listed axes of psi (mat's basis ordered like ``qubits``)."""
    k = len(qubits)
    m = mat.reshape((2,) * (2 * k))
    out = np.tensordot(m, psi, axes=(list(range(k, 2 * k)), list(qubits)))
    # tensordot puts the gate's output axes first; move them back to their qubit slots.
    return np.moveaxis(out, list(range(k)), list(qubits))


def state(circ: dict, replace: dict | None = None) -> np.ndarray:
    """Final state U|0^n> as an array of shape (2,)*n.

    ``replace`` maps a gate's index in ``circ["gates"]`` to a matrix used in its place
    (need not be unitary); the tests use it to build the state of one path of a cut."""
    n = circ["n_qubits"]
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for i in _ordered(circ):
        g = circ["gates"][i]
        m = replace[i] if replace and i in replace else G.matrix(g)
        psi = _apply(psi, m, g["qubits"])
    return psi


def amplitudes(circ: dict, bits: np.ndarray, open_qubits=()) -> np.ndarray:
    """Amplitudes for bit-strings ``bits`` [m, n]; with open qubits, [m, 2^n_open] where the
    batch index is big-endian over ``open_qubits`` in the order given (their bits in
    ``bits`` are ignored)."""
    psi = state(circ)
    bits = np.asarray(bits, dtype=np.int64)
    open_qubits = list(open_qubits)
    no = len(open_qubits)
    out = np.empty((bits.shape[0], 1 << no), dtype=np.complex128)
    for i, x in enumerate(bits):
        for j in range(1 << no):
            y = x.copy()
            for t, q in enumerate(open_qubits):
                y[q] = (j >> (no - 1 - t)) & 1
            out[i, j] = psi[tuple(y)]
    return out if no else out[:, 0]


def _adjoint(circ: dict, bits: np.ndarray, w: np.ndarray):
    """Adjoint sweep: for every fSim gate g (gate-list order)
    (sum_i w_i dpsi_i/dtheta_g, sum_i w_i dpsi_i/dphi_g) as complex arrays, the amplitudes
    psi_i, and sum_i w_i dpsi_i/dG_g[r, c] for every gate (keyed by gate index).

    The bra <Phi| = sum_i w_i <x_i| is carried backwards through the circuit while the ket
    is un-computed with each gate's inverse, so that at gate g the derivative of
    <Phi|U|0> with respect to that gate's matrix entries is the contraction of bra and ket
    over every other qubit.
    """
    n = circ["n_qubits"]
    bits = np.asarray(bits, dtype=np.int64)
    ket = state(circ)
    psi = np.array([ket[tuple(x)] for x in bits])
    bra = np.zeros((2,) * n, dtype=np.complex128)
    for wi, x in zip(w, bits):
        bra[tuple(x)] += wi
    fs_index = {}
    for i, g in enumerate(circ["gates"]):
        if g["kind"] == "fsim":
            fs_index[i] = len(fs_index)
    dth = np.zeros(len(fs_index), dtype=np.complex128)
    dph = np.zeros(len(fs_index), dtype=np.complex128)
    dgate = {}
    for i in reversed(_ordered(circ)):
        g = circ["gates"][i]
        m = G.matrix(g)
        q = g["qubits"]
        k = len(q)
        ket = _apply(ket, m.conj().T, q)  # undo the gate: ket = U_{<g}|0>
        rest = [a for a in range(n) if a not in q]
        b = np.transpose(bra, list(q) + rest).reshape(1 << k, -1)
        kk = np.transpose(ket, list(q) + rest).reshape(1 << k, -1)
        dmat = b @ kk.T  # d<Phi|..G..|ket>/dG[r, c] = sum_rest bra[r,rest] ket[c,rest]
        dgate[i] = dmat
        if g["kind"] == "fsim":
            j = fs_index[i]
            dth[j] = np.sum(dmat * G.dfsim_dtheta(g["theta"], g["phi"]))
            dph[j] = np.sum(dmat * G.dfsim_dphi(g["theta"], g["phi"]))
        bra = _apply(bra, m.T, q)  # bra <- bra . G  (row vector times matrix)
    return dth, dph, psi, dgate


def vjp_params(circ: dict, bits: np.ndarray, w: np.ndarray):
    """(sum_i w_i dpsi_i/dtheta_g, sum_i w_i dpsi_i/dphi_g) per fSim gate, and psi_i."""
    dth, dph, psi, _ = _adjoint(circ, bits, w)
    return dth, dph, psi


def vjp_gates(circ: dict, bits: np.ndarray, w: np.ndarray) -> dict:
    """sum_i w_i dpsi_i/dG_g[r, c] for every gate g (index in ``circ["gates"]``)."""
    return _adjoint(circ, bits, w)[3]


def linear_xeb(circ: dict, bits: np.ndarray) -> float:
    """Linear cross-entropy F = (2^n/m) sum_i |psi(x_i)|^2 - 1."""
    psi = amplitudes(circ, bits)
    n = circ["n_qubits"]
    return float((2.0 ** n) * np.mean(np.abs(psi) ** 2) - 1.0)


def linear_xeb_grad(circ: dict, bits: np.ndarray):
    """F and dF/d(theta, phi) for every fSim gate, as an [n_fsim, 2] real array."""
    n = circ["n_qubits"]
    m = len(bits)
    psi = amplitudes(circ, bits)
    scale = (2.0 ** n) / m
    # dF/dtheta = scale * sum_i 2 Re[conj(psi_i) dpsi_i/dtheta]
    dth, dph, _ = vjp_params(circ, bits, scale * np.conj(psi))
    grad = np.stack([2.0 * dth.real, 2.0 * dph.real], axis=1)
    return float(scale * np.sum(np.abs(psi) ** 2) - 1.0), grad


def identity_coupled_path_amplitudes(circ: dict, bits: np.ndarray, open_qubits=(), cuts=(),
                                     slice_id: int = 0) -> np.ndarray:
    """Closed form of one path of a circuit whose two-qubit gates are all the identity
    (fSim(0, 0), whose bond has two values, like CZ's).

    Such a circuit is a product state, and fixing the bonds of the cut links keeps it one:
    with the bond of the lower-id qubit q0 written as |k><k| and that of q1 as G_kk = I, a
    path is the product over qubits of <x_q| U_q |0>, where U_q is the qubit's one-qubit
    gates in time order with the projector |k_g><k_g| inserted at every cut gate g of which
    q is the lower-id qubit (k_g: that gate's digit of its link's value, earliest gate most
    significant; links in ``cuts`` order form the slice id, first most significant).
    Returns [m, 2^n_open] (batch index big-endian over ``open_qubits``)."""
    n = circ["n_qubits"]
    cuts = [tuple(sorted(c)) for c in cuts]
    link_gates = {c: [] for c in cuts}
    for i, g in sorted(enumerate(circ["gates"]), key=lambda t: t[1]["cycle"]):
        if len(g["qubits"]) == 2:
            if not np.allclose(G.matrix(g), np.eye(4), atol=0):
                raise ValueError("two-qubit gates must be the identity")
            key = tuple(sorted(g["qubits"]))
            if key in link_gates:
                link_gates[key].append(i)
    proj = {}  # gate index -> projector value on its lower-id qubit
    rem = int(slice_id)
    for c in reversed(cuts):
        gs = link_gates[c]
        v = rem % (1 << len(gs))
        rem >>= len(gs)
        for t, gi in enumerate(gs):
            proj[gi] = (v >> (len(gs) - 1 - t)) & 1
    vec = {q: np.array([1, 0], dtype=np.complex128) for q in range(n)}
    for i, g in sorted(enumerate(circ["gates"]), key=lambda t: t[1]["cycle"]):
        if len(g["qubits"]) == 1:
            q = g["qubits"][0]
            vec[q] = G.matrix(g) @ vec[q]
        elif i in proj:
            lo = min(g["qubits"])
            p = np.zeros((2, 2))
            p[proj[i], proj[i]] = 1
            vec[lo] = p @ vec[lo]
    open_qubits = list(open_qubits)
    no = len(open_qubits)
    out = np.empty((len(bits), 1 << no), dtype=np.complex128)
    for b, x in enumerate(np.asarray(bits)):
        base = np.prod([vec[q][int(x[q])] for q in range(n) if q not in open_qubits])
        for j in range(1 << no):
            v = base
            for t, q in enumerate(open_qubits):
                v = v * vec[q][(j >> (no - 1 - t)) & 1]
            out[b, j] = v
    return out
