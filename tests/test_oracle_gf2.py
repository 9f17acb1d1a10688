"""Pins of the GF(2) closed form for CZ-only circuits (oracle/gf2.py): the exponential sum of
a quadratic form against brute force, and per-path amplitudes against the two FP64 engines
(E2 per path, E1 for the sum over paths)."""
import itertools

import numpy as np
import pytest

import rqc_inputs as R
from oracle import gf2
from oracle import statevector as E1
from oracle import tn as E2


def _brute(n, pairs, linear, const, fixed):
    s = 0
    for y in itertools.product((0, 1), repeat=n):
        if any(y[i] != v for i, v in fixed.items()):
            continue
        e = const + sum(l * yi for l, yi in zip(linear, y)) + sum(y[a] * y[b] for a, b in pairs)
        s += (-1) ** (e % 2)
    return s


@pytest.mark.parametrize("seed", range(40))
def test_quadratic_sum_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 11))
    pairs = [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(int(rng.integers(0, 3 * n)))]
    linear = [int(v) for v in rng.integers(0, 2, n)]
    const = int(rng.integers(0, 2))
    fixed = {int(i): int(rng.integers(0, 2)) for i in rng.choice(n, int(rng.integers(0, n)), replace=False)}
    assert gf2.quadratic_sum(n, pairs, linear, const, fixed) == _brute(n, pairs, linear, const, fixed)


def test_cz_only_paths_match_fp64_engines():
    """3x4 CZ-only circuit (3 CZ per link at depth 1+24+1: an even count would cancel), two cut
    links, a 2-qubit open batch: every path against E2's sliced contraction, and the sum over
    paths against E1."""
    c = R.without_kinds(R.grid_rqc(3, 4, 24, 5), ("x12", "y12", "t"))
    op = [11, 7]
    bits = R.bitstrings(12, 6, 21, op)
    cuts = [(5, 6), (2, 6)]
    S = E2.num_slices(c, cuts)
    assert S == 64
    total = np.zeros((6, 4))
    nonzero = 0
    for sid in range(S):
        got = gf2.cz_only_slice_amplitudes(c, bits, op, cuts, sid)
        want = E2.amplitudes(c, bits, op, cuts=cuts, slice_ids=[sid])
        assert np.allclose(got, want, atol=1e-13), sid
        nonzero += bool(np.abs(want).max() > 1e-12)
        total += got
    assert 0 < nonzero < S  # paths whose gates' k differ vanish
    full = E1.amplitudes(c, bits, op)
    assert np.allclose(total, full, atol=1e-13)
    assert np.allclose(gf2.cz_only_slice_amplitudes(c, bits, op), full, atol=1e-13)
