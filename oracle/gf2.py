"""Exact amplitudes of CZ-only circuits at any size, per path of a cut (slice).  TEST
INFRASTRUCTURE (see ``oracle/__init__.py``).

A circuit made of a layer of H on every qubit, CZ gates only, and a final layer of H is
diagonal between the two H layers, so (Methods B's tensor network, evaluated in closed form)

    psi(x) = 2^-n  sum over y in {0,1}^n  (-1)^( x.y + sum over CZ gates (a, b) of y_a y_b ),

an exponential sum of a quadratic form over GF(2).  Such a sum is 0 or +-2^k and is computed
exactly by eliminating variables two at a time: summing over y_i, whose terms are
y_i (l_i + sum over its quadratic partners y_k), gives 2 when that linear form vanishes and 0
otherwise; the constraint is solved for one partner y_j and substituted into the rest.

Per path (Methods B.1, cutting indexes): a CZ splits along the elementary basis of its
lower-id qubit q0 as sum_k |k><k| (x) Z^k.  Fixing the bond of a cut link fixes the k of each
of its r gates; since q0's computational value y_q0 is constant between the H layers, a path
is non-zero only when all r values equal one v, and it then contributes the terms with
y_q0 = v and (-1)^(r v y_q1) in place of the link's r CZ gates.  The bond value of a link is
the mixed radix of its gates' k, earliest gate most significant; a slice id is the mixed radix
of the cut links' values, first cut most significant.
"""
from __future__ import annotations

import numpy as np


def quadratic_sum(n: int, pairs, linear, const: int = 0, fixed=None) -> int:
    """sum over y in {0,1}^n with y_i = fixed[i] (i in fixed) of
    (-1)^(const + linear.y + sum over (a, b) in pairs of y_a y_b), exactly (a Python int).
    ``pairs`` may repeat a pair (terms add mod 2); a pair (a, a) is the linear term y_a."""
    A = np.zeros((n, n), dtype=bool)
    lin = np.zeros(n, dtype=bool)
    lin[:] = np.asarray(linear, dtype=np.int64).reshape(n) % 2 == 1
    c = const % 2
    for a, b in pairs:
        if a == b:
            lin[a] ^= True
        else:
            A[a, b] ^= True
            A[b, a] ^= True
    alive = np.ones(n, dtype=bool)
    # fixed variables: y_i = v turns y_i y_j into v y_j and l_i y_i into a constant
    for i, v in (fixed or {}).items():
        v = int(v) & 1
        if v:
            lin ^= A[i]
            c ^= int(lin[i])
        A[i, :] = False
        A[:, i] = False
        lin[i] = False
        alive[i] = False
    power = 0
    while alive.any():
        i = int(np.flatnonzero(alive)[0])
        nb = np.flatnonzero(A[i] & alive)
        if nb.size == 0:
            # y_i appears only linearly: the sum over it is 2 or 0
            if lin[i]:
                return 0
            power += 1
            alive[i] = False
            lin[i] = False
            continue
        # sum over y_i: 2 when y_j = l_i + sum over the other partners k of y_k, else 0
        j = int(nb[0])
        rest = nb[1:]
        li = bool(lin[i])
        # y_i leaves the form
        A[i, :] = False
        A[:, i] = False
        lin[i] = False
        alive[i] = False
        # substitute y_j: its linear term l_j y_j and its quadratic terms y_j y_m
        lj = bool(lin[j])
        if lj:
            c ^= int(li)
            for k in rest:
                lin[k] ^= True
        partners = A[j] & alive
        if li:
            lin ^= partners
        # sum over k in rest and m in partners of y_k y_m: a term with k = m is linear
        # (y_k y_k = y_k); a pair met in both orders cancels
        in_rest = np.zeros(n, dtype=bool)
        in_rest[rest] = True
        lin ^= in_rest & partners
        M = np.outer(in_rest, partners)
        np.fill_diagonal(M, False)
        A ^= M ^ M.T
        A[j, :] = False
        A[:, j] = False
        lin[j] = False
        alive[j] = False
        power += 1
    return (-1) ** c * 2 ** power


def _cz_structure(circ: dict):
    n = int(circ["n_qubits"])
    gates = sorted(circ["gates"], key=lambda g: g["cycle"])
    last = max(g["cycle"] for g in gates)
    first_h = {g["qubits"][0] for g in gates if g["kind"] == "h" and g["cycle"] == 0}
    last_h = {g["qubits"][0] for g in gates if g["kind"] == "h" and g["cycle"] == last}
    if first_h != set(range(n)) or last_h != set(range(n)):
        raise ValueError("needs a layer of H first and last")
    links = {}
    for g in gates:
        if g["kind"] == "h" and g["cycle"] in (0, last):
            continue
        if g["kind"] != "cz":
            raise ValueError("only CZ gates between the H layers (got %s)" % g["kind"])
        a, b = sorted(g["qubits"])
        links.setdefault((a, b), 0)
        links[(a, b)] += 1
    return n, links


def cz_only_slice_amplitudes(circ: dict, bits, open_qubits=(), cuts=(), slice_id=None):
    """Amplitudes [m, 2^n_open] (real, exact up to the final scaling by 2^-n) of a CZ-only
    circuit for bit-strings ``bits`` [m, n] (open qubits' entries ignored; the batch index is
    big-endian over ``open_qubits``), summed over the paths of ``cuts`` ((lo, hi) links, first
    most significant) or, with ``slice_id``, for that one path."""
    n, links = _cz_structure(circ)
    bits = np.asarray(bits, dtype=np.int64).reshape(-1, n)
    open_qubits = list(open_qubits)
    cut_links = [tuple(sorted(c)) for c in cuts]
    fixed, extra = {}, []
    pairs = [l for l, r in links.items() if l not in cut_links for _ in range(r % 2)]
    if slice_id is not None:
        # the slice's value on each cut link, least significant cut last
        rem = int(slice_id)
        vals = []
        for l in reversed(cut_links):
            r = links[l]
            vals.append(rem & ((1 << r) - 1))
            rem >>= r
        vals.reverse()
        for (lo, hi), val in zip(cut_links, vals):
            r = links[(lo, hi)]
            if val not in (0, (1 << r) - 1):  # the gates' k differ: the path vanishes
                return np.zeros((bits.shape[0], 1 << len(open_qubits)))
            v = 1 if val else 0
            if lo in fixed and fixed[lo] != v:
                return np.zeros((bits.shape[0], 1 << len(open_qubits)))
            fixed[lo] = v
            if v and r % 2:
                extra.append((hi, hi))  # (-1)^(r v y_hi): a linear term on hi
    else:
        pairs += [l for l in cut_links for _ in range(links[l] % 2)]
    out = np.zeros((bits.shape[0], 1 << len(open_qubits)))
    for b, x in enumerate(bits):
        for o in range(1 << len(open_qubits)):
            xx = x.copy()
            for t, q in enumerate(open_qubits):
                xx[q] = (o >> (len(open_qubits) - 1 - t)) & 1
            s = quadratic_sum(n, pairs + extra, xx, 0, fixed)
            out[b, o] = s / 2.0 ** n
    return out
