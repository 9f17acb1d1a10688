"""Error measures used to compare results.  TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Amplitudes are compared after scaling by 2^(n/2), so that a typical amplitude has modulus
about one.  Per-element error |s - s_ref| / max(|s_ref|, rms(s_ref)): the rms floor keeps
the tiny amplitudes in the Porter-Thomas tail from dominating.  Gradients are compared by
relative L2 norm.  Both sides are flattened; they must hold the same number of elements
(a size mismatch raises instead of broadcasting one side over the other).
"""
from __future__ import annotations

import numpy as np


def _flat_pair(a, b, dtype):
    a = np.asarray(a, dtype=dtype).ravel()
    b = np.asarray(b, dtype=dtype).ravel()
    if a.size != b.size:
        raise ValueError("compared arrays differ in size: %d vs %d" % (a.size, b.size))
    return a, b


def amp_errors(amps, ref, n_qubits: int) -> dict:
    s, r = _flat_pair(amps, ref, np.complex128)
    s = s * 2.0 ** (n_qubits / 2)
    r = r * 2.0 ** (n_qubits / 2)
    rms = float(np.sqrt(np.mean(np.abs(r) ** 2))) if r.size else 0.0
    den = np.maximum(np.abs(r), rms if rms > 0 else 1.0)
    e = np.abs(s - r) / den
    l2 = float(np.linalg.norm(s - r) / max(np.linalg.norm(r), 1e-300))
    return {"max": float(e.max()) if e.size else 0.0,
            "median": float(np.median(e)) if e.size else 0.0,
            "l2": l2}


def rel_l2(a, b) -> float:
    a, b = _flat_pair(a, b, np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
