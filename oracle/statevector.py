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
