"""Pins of the frugal-sampling oracle (Methods, "Fast sampling technique" and "Sampling from a
non fully-thermalized Porter-Thomas distribution") against the paper's printed numbers,
Porter-Thomas closed forms checked by Monte Carlo, the exact law of the first acceptance, and
special cases."""
import math
import os

import numpy as np

import rqc_inputs as R
from oracle import sampling as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_batch_acceptance_reproduces_the_printed_numbers():
    rows = [l.split() for l in open(os.path.join(GOLD, "frugal_acceptance_c2.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for m, nc, acc, batches in rows:
        p = S.batch_acceptance(float(m), int(nc))
        assert abs(p - float(acc)) < 6e-5
        assert abs(1e6 / p - float(batches)) / float(batches) < 2e-3


def test_acceptance_under_porter_thomas_by_monte_carlo():
    """Synthetic Porter-Thomas batches: the empirical share of batches that yield a bit-string
    matches 1 - (1 - E[min(1, x/M)])^N_C, and, to O(e^-M), the paper's 1 - (1 - 1/M)^N_C."""
    n_q, nb, blen = 20, 20000, 64
    amps = R.porter_thomas_amplitudes(nb, blen, n_q, 11)
    for m, nc in ((3.0, 4), (10.0, 8)):
        order, u = R.sampling_draws(nb, blen, nc, 12 + int(m))
        got = S.frugal_sample(amps, order, u, n_q, m)
        rate = np.mean(np.array(got) >= 0)
        want = S.porter_thomas_acceptance(m, nc)
        sigma = math.sqrt(want * (1 - want) / nb)
        assert abs(rate - want) < 4 * sigma, (m, rate, want)
        assert abs(S.batch_acceptance(m, nc) - want) < 2 * nc * math.exp(-m) / m
        # an accepted value is one that was visited
        for b in range(0, nb, 997):
            assert got[b] == -1 or got[b] in set(order[b].tolist())


def test_tail_error_matches_the_porter_thomas_closed_form():
    """E[x 1(x > M)] = (M + 1) e^-M for x ~ Exp(1); the estimate over 1.28M synthetic amplitudes
    lands within 4 standard errors (variance from E[x^2 1(x > M)] = (M^2 + 2M + 2) e^-M)."""
    n_q, nb, blen = 24, 20000, 64
    amps = R.porter_thomas_amplitudes(nb, blen, n_q, 21)
    n = nb * blen
    for m in (3.0, 10.0):
        got = S.tail_error(amps, n_q, m)
        want = S.porter_thomas_tail(m)
        var = (m * m + 2 * m + 2) * math.exp(-m) - want * want
        assert abs(got - want) < 4 * math.sqrt(var / n), (m, got, want)
    assert abs(S.porter_thomas_tail(10.0) - 5.0e-4) < 5e-6  # the value the paper calls 1e-4 order


def test_first_acceptance_follows_the_product_law():
    """For one batch visited in a fixed order, the first acceptance is at visit j with
    probability a_j prod_{i<j} (1 - a_i), a_i = min(1, N p_i / M), and no acceptance with
    prod_i (1 - a_i)."""
    n_q, m = 4, 4.0
    dim = 2.0 ** n_q
    a = np.array([0.03, 0.1, 0.35, 0.05, 0.2]) ** 0.5 * np.exp(1j * np.arange(5))
    acc = np.minimum(1.0, dim * np.abs(a) ** 2 / m)
    law = [acc[j] * np.prod(1 - acc[:j]) for j in range(5)] + [np.prod(1 - acc)]
    trials = 40000
    rng = np.random.Generator(np.random.PCG64(5))
    u = rng.random((trials, 5))
    order = np.tile(np.arange(5, dtype=np.int32), (trials, 1))
    got = S.frugal_sample([a] * trials, order, u, n_q, m)
    counts = np.bincount([5 if g < 0 else g for g in got], minlength=6) / trials
    for j in range(6):
        assert abs(counts[j] - law[j]) < 4 * math.sqrt(law[j] * (1 - law[j]) / trials) + 1e-12


def test_special_cases():
    n_q, m = 6, 10.0
    big = np.full((3, 8), math.sqrt(20.0 / 2 ** n_q), dtype=complex)  # N p = 20 > M everywhere
    order, u = R.sampling_draws(3, 8, 5, 3)
    assert S.frugal_sample(big, order, u, n_q, m) == [int(o[0]) for o in order]
    zero = np.zeros((3, 8), dtype=complex)
    assert S.frugal_sample(zero, order, u, n_q, m) == [-1, -1, -1]
    # u = 0 accepts the first visited value of non-zero probability
    amps = np.zeros((1, 8), dtype=complex)
    amps[0, 6] = 1e-9j
    assert S.frugal_sample(amps, [[2, 6, 1]], [[0.0, 0.0, 0.0]], n_q, m) == [6]
    # p is re*re + im*im, each step rounded once
    z = complex(0.1, 0.3)
    assert S.probability(z) == 0.1 * 0.1 + 0.3 * 0.3
    assert abs(S.tail_error(big, n_q, m) - 20.0) < 1e-12


def test_sampling_draws_are_random_subsets_in_random_order():
    order, u = R.sampling_draws(4000, 16, 5, 77)
    assert order.shape == (4000, 5) and order.dtype == np.int32 and u.shape == (4000, 5)
    assert all(len(set(r.tolist())) == 5 for r in order)
    assert order.min() >= 0 and order.max() < 16 and 0 <= u.min() and u.max() < 1
    # every value equally likely at every visit position (chi-square, 15 dof, far tail)
    for j in range(5):
        c = np.bincount(order[:, j], minlength=16)
        chi2 = np.sum((c - 250.0) ** 2 / 250.0)
        assert chi2 < 45.0, (j, chi2)


def test_fidelity_samples_mix_exact_and_uniform_samples():
    """Fraction of perfect fidelity amplitudes: a share f of the batches gives exact samples
    (closed bits kept, the accepted open value written big-endian into the open qubits), the
    rest give their uniform bit-string; an exact batch that accepts nothing gives no sample."""
    n_q, blen, nb, m = 10, 8, 20000, 10.0
    op = [7, 2, 9]
    rng = np.random.Generator(np.random.PCG64(31))
    closed = rng.integers(0, 2, (nb, n_q))
    closed[:, op] = 0
    uniform = rng.integers(0, 2, (nb, n_q))
    coins = rng.random(nb)
    amps = R.porter_thomas_amplitudes(nb, blen, n_q, 32)
    order, u = R.sampling_draws(nb, blen, blen, 33)
    for f in (0.0, 0.01, 0.25, 1.0):
        samples, status = S.fidelity_samples(amps, closed, op, coins, uniform, order, u, n_q, m, f)
        status = np.array(status)
        exact = coins < f
        assert np.array_equal(status != 0, exact)
        # an exact batch is exhausted as often as the batch acceptance law says
        if exact.sum() > 100:
            miss = np.mean(status[exact] == -1)
            want = 1 - S.porter_thomas_acceptance(m, blen)
            assert abs(miss - want) < 4 * math.sqrt(want * (1 - want) / exact.sum()) + 1e-3
        picks = S.frugal_sample(amps, order, u, n_q, m)
        for b in range(0, nb, 37):
            if status[b] == 0:
                assert samples[b] == uniform[b].tolist()
            elif status[b] == 1:
                x = samples[b]
                assert [x[q] for q in range(n_q) if q not in op] == \
                    [int(closed[b][q]) for q in range(n_q) if q not in op]
                assert x[op[0]] * 4 + x[op[1]] * 2 + x[op[2]] == picks[b]
            else:
                assert samples[b] is None and picks[b] == -1
