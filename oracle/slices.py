"""Seeded choice of a fraction of the paths.  TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

The paper sums a randomly chosen fraction f of the paths to obtain fidelity-f amplitudes
(Methods C.1).  Reading used for the random choice, so that both sides can draw the same
subset from a seed: k = f * S must be an integer >= 1; shuffle [0, S) with Fisher-Yates
(i from S-1 down to 1, j = next() mod (i + 1), swap a[i], a[j]) driven by SplitMix64
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014:
state += 0x9E3779B97F4A7C15; z = state; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31), keep the first k entries, sorted.

Block mode (a reuse-friendly variant of the same fraction): k must divide S; the subset is
the k consecutive ids [j k, (j + 1) k) with j = next() mod (S / k) from SplitMix64(seed).
Slice ids are mixed radix over the cuts, first cut most significant, so with S and k powers
of two a block fixes the leading cuts' values and runs over all values of the trailing ones.
"""
from __future__ import annotations

M64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & M64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)


def count_for_fidelity(total: int, fidelity: float) -> int:
    k = fidelity * total
    ki = int(round(k))
    if not (0.0 < fidelity <= 1.0) or abs(k - ki) > 1e-9 * max(1.0, k) or ki < 1:
        raise ValueError("fidelity * slices must be an integer >= 1")
    return ki


def select(total: int, fidelity: float, seed: int) -> list[int]:
    k = count_for_fidelity(total, fidelity)
    a = list(range(total))
    g = SplitMix64(seed)
    for i in range(total - 1, 0, -1):
        j = g.next() % (i + 1)
        a[i], a[j] = a[j], a[i]
    return sorted(a[:k])


def select_block(total: int, fidelity: float, seed: int) -> list[int]:
    k = count_for_fidelity(total, fidelity)
    if total % k:
        raise ValueError("block slice subsets need fidelity * slices to divide the slices")
    j = SplitMix64(seed).next() % (total // k)
    return list(range(j * k, (j + 1) * k))
