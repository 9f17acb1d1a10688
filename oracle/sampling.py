"""Fast frugal rejection sampling over open-qubit batches.  TEST INFRASTRUCTURE (see
``oracle/__init__.py``).

The paper's fast sampling technique (Methods, "Fast sampling technique") draws one output
bit-string per batch of amplitudes that share the bit-string of the closed qubits: N_C of the
batch's open-qubit values are chosen at random without repetition and visited in a random
order; the visited bit-string s is accepted with probability min(1, N p(s) / M), with
p(s) = |psi(s)|^2 and N = 2^n the Hilbert-space dimension, and the batch ends at its first
acceptance (at most one bit-string per batch) or when its N_C values are used up.

Random numbers are inputs: ``order[b]`` lists the batch's N_C visited values in visiting
order (a random subset without repetition, already shuffled), ``u[b][j]`` is the uniform
number in [0, 1) drawn for the j-th visit.  Acceptance with probability a is read as u < a;
with a = min(1, N p / M) and u < 1 this is u * M < N * p, the form used here (N * p is exact for
N a power of two, so the decision is one rounding of u * M against an exactly scaled p).

Fidelity-f samples by the Results' second method ("Fraction of perfect fidelity amplitudes"):
the state f |psi><psi| + (1 - f) I / N is sampled by taking, per batch, an exact sample with
probability f (the batch's amplitudes at full fidelity through the sampler above) and a
uniformly random bit-string otherwise.  The coin per batch and the uniform bit-strings are
inputs, like the sampler's random numbers.

The same section gives the acceptance probability of a batch under Porter-Thomas statistics,
1 - (1 - 1/M)^N_C, and the sampling error estimate of the next section (Methods, "Sampling
from a non fully-thermalized Porter-Thomas distribution"): the sum of N p over the computed
amplitudes with p > M / N, divided by the number of amplitudes computed.
"""
from __future__ import annotations

import math


def probability(amp: complex) -> float:
    """|amp|^2 as re*re + im*im, each operation rounded once (no fused multiply-add)."""
    re, im = float(amp.real), float(amp.imag)
    return re * re + im * im


def frugal_sample(amps, order, u, n_qubits: int, m: float) -> list[int]:
    """One accepted open-qubit value per batch, or -1 when the batch is exhausted.

    amps[b][s]: amplitude of batch b's bit-string with open-qubit value s; order[b][j] and
    u[b][j] as in the module docstring.
    """
    dim = 2.0 ** n_qubits
    out = []
    for b in range(len(amps)):
        pick = -1
        for j in range(len(order[b])):
            s = int(order[b][j])
            if float(u[b][j]) * m < dim * probability(amps[b][s]):
                pick = s
                break
        out.append(pick)
    return out


def tail_error(amps, n_qubits: int, m: float) -> float:
    """Sampling error estimate: sum over all computed amplitudes of N p where N p > M, divided
    by the number of amplitudes."""
    dim = 2.0 ** n_qubits
    total, count = 0.0, 0
    for batch in amps:
        for a in batch:
            x = dim * probability(a)
            if x > m:
                total += x
            count += 1
    return total / count


def batch_acceptance(m: float, n_c: int) -> float:
    """The paper's probability that a batch of N_C visits yields a bit-string."""
    return 1.0 - (1.0 - 1.0 / m) ** n_c


def porter_thomas_acceptance(m: float, n_c: int) -> float:
    """The same for N p exactly exponential: one visit accepts with probability
    E[min(1, x / M)] = (1 - e^-M) / M, x ~ Exp(1)."""
    q = (1.0 - math.exp(-m)) / m
    return 1.0 - (1.0 - q) ** n_c


def porter_thomas_tail(m: float) -> float:
    """E[x 1(x > M)] = (M + 1) e^-M for x ~ Exp(1): the error estimate's Porter-Thomas value."""
    return (m + 1.0) * math.exp(-m)


def fidelity_samples(exact_amps, closed_bits, open_qubits, coins, uniform_bits, order, u,
                     n_qubits: int, m: float, fidelity: float):
    """Per batch b: status 1 and the exact sample (closed_bits[b] with the accepted open value
    written into open_qubits, the first open qubit most significant) when coins[b] < f and the
    batch accepts a value; status -1 and no sample when coins[b] < f but none is accepted; status
    0 and uniform_bits[b] otherwise.  exact_amps[b] holds batch b's amplitudes and is read only
    where coins[b] < f."""
    no = len(open_qubits)
    samples, status = [], []
    for b in range(len(coins)):
        if float(coins[b]) < fidelity:
            pick = frugal_sample([exact_amps[b]], [order[b]], [u[b]], n_qubits, m)[0]
            if pick < 0:
                samples.append(None)
                status.append(-1)
                continue
            x = [int(v) for v in closed_bits[b]]
            for t, q in enumerate(open_qubits):
                x[q] = (pick >> (no - 1 - t)) & 1
            samples.append(x)
            status.append(1)
        else:
            samples.append([int(v) for v in uniform_bits[b]])
            status.append(0)
    return samples, status
