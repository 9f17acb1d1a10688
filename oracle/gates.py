"""Gate matrices for the oracle (FP64).  TEST INFRASTRUCTURE: only tests, the smoke check and
the CPU-baseline leg of the benchmark may use anything under ``oracle/``.

The paper names the gates (Methods A) but prints only iSWAP.  Readings used here:
  H      = (1/sqrt2) [[1, 1], [1, -1]]
  X^1/2  = 1/2 [[1+i, 1-i], [1-i, 1+i]]
  Y^1/2  = 1/2 [[1+i, -1-i], [1+i, 1+i]]
  T      = diag(1, e^{i pi/4})
  CZ     = diag(1, 1, 1, -1)
  fSim(theta, phi) = [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,e^{-i phi}]]
Two-qubit matrices are in the basis |q0 q1> = 00, 01, 10, 11 with q0 the first listed qubit.
fSim(-pi/2, 0) is the paper's iSWAP (Methods A), fSim(0, pi) is CZ and fSim(0, 0) is the
identity; the tests pin these special cases.
"""
from __future__ import annotations

import numpy as np

_S2 = 1.0 / np.sqrt(2.0)

H = np.array([[_S2, _S2], [_S2, -_S2]], dtype=np.complex128)
X12 = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
Y12 = 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128)
T = np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)

ONE_QUBIT = {"h": H, "x12": X12, "y12": Y12, "t": T}


def fsim(theta: float, phi: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


def dfsim_dtheta(theta: float, phi: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[0, 0, 0, 0],
                     [0, -s, -1j * c, 0],
                     [0, -1j * c, -s, 0],
                     [0, 0, 0, 0]], dtype=np.complex128)


def dfsim_dphi(theta: float, phi: float) -> np.ndarray:
    m = np.zeros((4, 4), dtype=np.complex128)
    m[3, 3] = -1j * np.exp(-1j * phi)
    return m


def matrix(g: dict) -> np.ndarray:
    """Matrix of one gate of the circuit format (basis ordered by g["qubits"])."""
    k = g["kind"]
    if k in ONE_QUBIT:
        return ONE_QUBIT[k]
    if k == "cz":
        return CZ
    if k == "fsim":
        return fsim(g["theta"], g["phi"])
    raise ValueError("unknown gate kind %r" % k)
