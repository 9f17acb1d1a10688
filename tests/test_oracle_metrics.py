"""Pins of the error measures every parity check rests on, on vectors whose errors are worked
out by hand (the values below are not produced by the code under test)."""
import numpy as np
import pytest

from oracle import metrics


# Reference (already scaled, n_qubits = 0): moduli 3, 4, 0, 0, so rms = sqrt(25 / 4) = 2.5.
# Result differs by 0.3 on the first element, 0.5 on the third (a zero reference value, where
# the rms floor decides the denominator) and not at all elsewhere.
REF = np.array([3.0, 4.0j, 0.0, 0.0])
GOT = np.array([3.3, 4.0j, 0.5, 0.0])
# per element: 0.3 / max(3, 2.5) = 0.1; 0 / 4 = 0; 0.5 / max(0, 2.5) = 0.2; 0
E_MAX, E_MEDIAN = 0.2, 0.05        # median of {0, 0, 0.1, 0.2} = (0 + 0.1) / 2
E_L2 = np.sqrt(0.3 ** 2 + 0.5 ** 2) / 5.0   # |ref| = sqrt(9 + 16) = 5


def test_amp_errors_hand_computed():
    e = metrics.amp_errors(GOT, REF, 0)
    assert e["max"] == pytest.approx(E_MAX, rel=1e-12)
    assert e["median"] == pytest.approx(E_MEDIAN, rel=1e-12)
    assert e["l2"] == pytest.approx(E_L2, rel=1e-12)
    # the floor is the reference's rms: over the result it would give 0.5 / 2.6048 = 0.192
    assert e["max"] != pytest.approx(0.5 / np.sqrt(np.mean(np.abs(GOT) ** 2)), rel=1e-6)


def test_amp_errors_relative_measures_ignore_the_scale():
    # amplitudes of an n = 4 qubit circuit are 2^-2 times the scaled values
    e = metrics.amp_errors(GOT / 4.0, REF / 4.0, 4)
    assert e["max"] == pytest.approx(E_MAX, rel=1e-12)
    assert e["median"] == pytest.approx(E_MEDIAN, rel=1e-12)
    assert e["l2"] == pytest.approx(E_L2, rel=1e-12)


def test_amp_errors_shapes():
    # a [m, 1] column against an [m] vector compares element by element
    e = metrics.amp_errors(GOT[:, None], REF, 0)
    assert e["max"] == pytest.approx(E_MAX, rel=1e-12)
    # different element counts never broadcast (a [64] batch against one amplitude)
    with pytest.raises(ValueError):
        metrics.amp_errors(np.ones(64), np.ones(1), 0)
    with pytest.raises(ValueError):
        metrics.amp_errors(np.ones((4, 2)), np.ones(4), 0)


def test_amp_errors_exact_and_all_zero_reference():
    e = metrics.amp_errors(REF, REF, 7)
    assert e == {"max": 0.0, "median": 0.0, "l2": 0.0}
    # zero reference: the floor falls back to 1, so the error is the result's modulus
    e = metrics.amp_errors(np.array([0.0, 0.25j]), np.zeros(2), 0)
    assert e["max"] == pytest.approx(0.25) and e["median"] == pytest.approx(0.125)


def test_rel_l2_hand_computed():
    # |a - b| = |(0, 2, 2)| = sqrt(8), |b| = 1
    assert metrics.rel_l2([1.0, 2.0, 2.0], [1.0, 0.0, 0.0]) == pytest.approx(np.sqrt(8.0))
    # complex: a - b = (4j, -4j), |b| = |(3, 4j)| = 5
    assert metrics.rel_l2([3 + 4j, 0.0], [3.0, 4j]) == pytest.approx(np.sqrt(32.0) / 5.0)
    assert metrics.rel_l2(np.arange(6.0).reshape(2, 3), np.arange(6.0)) == 0.0
    with pytest.raises(ValueError):
        metrics.rel_l2(np.ones(3), np.ones(1))
