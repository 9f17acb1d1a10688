"""Seeded synthetic inputs: random quantum circuits (RQCs) on 2D layouts and output bit-strings.

This module is shared by the CPU oracle and the HIP path as *input data only*: it decides
which gate kind sits where and with which angles, never what a gate's matrix is or how a
circuit is simulated.  Each consumer turns gate kinds into matrices with code of its own.

Circuit prescription (paper, Methods A, rules (1)-(5) and the revised-RQC remarks):
  cycle 0       Hadamard on every qubit;
  cycles 1..t   two-qubit gates on the couplers of layer ``(c-1) mod 8`` of an eight-layer
                cover of the lattice; a qubit idle in cycle c that was in a two-qubit gate
                in cycle c-1 gets X^1/2 or Y^1/2 with probability 1/2 each; a qubit idle in
                cycle c whose gate in cycle c-1 was X^1/2, Y^1/2 or H gets T;
  cycle t+1     Hadamard on every qubit.
The figure that fixes the eight coupler layers is not legible in the paper, so the layers
are read as: horizontal bond (r,c)-(r,c+1) belongs to H[c mod 2][r mod 2], vertical bond
(r,c)-(r+1,c) to V[r mod 2][c mod 2], cycled in the order H00 V00 H11 V11 H01 V01 H10 V10
(never two horizontal or two vertical layers in a row, as the revised rules require; every
layer is a matching and every link is used exactly once per eight cycles).

Circuit format (plain dict, JSON-serialisable)::

    {"n_qubits": n, "xy": [[r, c], ...], "depth": t,
     "gates": [{"cycle": c, "kind": "h"|"x12"|"y12"|"t"|"cz"|"fsim",
                "qubits": [a] or [a, b], "theta": float, "phi": float}, ...]}

Qubit ids are row-major over the layout.  ``theta``/``phi`` are present for ``fsim`` only.
"""
from __future__ import annotations

import json
import math

import numpy as np

LAYER_ORDER = ("H00", "V00", "H11", "V11", "H01", "V01", "H10", "V10")

ONE_QUBIT_KINDS = ("h", "x12", "y12", "t")
TWO_QUBIT_KINDS = ("cz", "fsim")


# ----------------------------------------------------------------------------- layouts
def grid_layout(rows: int, cols: int) -> list[list[int]]:
    """Row-major coordinates of a rows x cols square grid."""
    return [[r, c] for r in range(rows) for c in range(cols)]


def diamond_layout() -> list[list[int]]:
    """The 70-qubit diamond lattice (72-site Bristlecone-like layout minus its two corners).

    Sites sit in 12 rows of 6; site (row, k) has square-grid coordinates with
    x - y = row and x + y = 2k + (row mod 2), so each site couples to up to four sites in
    the neighbouring rows.  The two sites with a single neighbour, (0, 0) and (11, 5), are
    removed, which the paper notes costs nothing (Methods B.1, Bristlecone-72 -> -70).
    Returned coordinates are (x, y - min y), sorted row-major.
    """
    pts = []
    for row in range(12):
        for k in range(6):
            if (row, k) in ((0, 0), (11, 5)):
                continue
            s = 2 * k + (row % 2)
            x = (row + s) // 2
            y = (s - row) // 2
            pts.append((x, y))
    ymin = min(p[1] for p in pts)
    pts = sorted((x, y - ymin) for x, y in pts)
    return [list(p) for p in pts]


def couplers(xy) -> list[tuple[int, int]]:
    """All unit-distance pairs (a, b), a < b, sorted."""
    pos = {tuple(p): i for i, p in enumerate(xy)}
    out = []
    for i, (r, c) in enumerate(xy):
        for dr, dc in ((0, 1), (1, 0)):
            j = pos.get((r + dr, c + dc))
            if j is not None:
                out.append((min(i, j), max(i, j)))
    return sorted(out)


def layer_of(xy, a: int, b: int) -> int:
    """Index (0..7, position in LAYER_ORDER) of the layer that holds coupler (a, b)."""
    (r0, c0), (r1, c1) = sorted([tuple(xy[a]), tuple(xy[b])])
    if r0 == r1:  # horizontal (r, c)-(r, c+1)
        name = "H%d%d" % (c0 % 2, r0 % 2)
    else:  # vertical (r, c)-(r+1, c)
        name = "V%d%d" % (r0 % 2, c0 % 2)
    return LAYER_ORDER.index(name)


# ----------------------------------------------------------------------------- circuits
def rqc(xy, depth: int, seed: int, two_qubit: str = "cz", theta: float = math.pi / 2,
        phi: float = math.pi / 6, jitter_sd: float = 0.0, jitter_seed: int | None = None,
        name: str = "") -> dict:
    """Random circuit of depth 1+depth+1 on layout ``xy`` (rules listed in the module doc).

    Single-qubit choices draw from numpy PCG64(seed): one draw of integers(0, 2) per qubit
    that needs X^1/2 / Y^1/2, cycles ascending, qubits by id (0 -> X^1/2, 1 -> Y^1/2).
    For ``two_qubit="fsim"`` each gate's angles are theta + e1, phi + e2 with e1, e2 drawn
    (in gate order, theta first) from N(0, jitter_sd^2) under PCG64(jitter_seed).
    """
    if two_qubit not in TWO_QUBIT_KINDS:
        raise ValueError("two_qubit must be one of %r" % (TWO_QUBIT_KINDS,))
    n = len(xy)
    cps = couplers(xy)
    by_layer = [[] for _ in range(8)]
    for a, b in cps:
        by_layer[layer_of(xy, a, b)].append((a, b))
    rng = np.random.Generator(np.random.PCG64(seed))
    jrng = np.random.Generator(np.random.PCG64(seed if jitter_seed is None else jitter_seed))
    gates = [{"cycle": 0, "kind": "h", "qubits": [q]} for q in range(n)]
    prev = ["h"] * n  # kind of the gate each qubit saw in the previous cycle ("" = none)
    for cyc in range(1, depth + 1):
        layer = by_layer[(cyc - 1) % 8]
        busy = [False] * n
        cur = [""] * n
        for a, b in layer:
            g = {"cycle": cyc, "kind": two_qubit, "qubits": [a, b]}
            if two_qubit == "fsim":
                e1, e2 = (jrng.normal(0.0, jitter_sd, 2) if jitter_sd > 0 else (0.0, 0.0))
                g["theta"] = float(theta + e1)
                g["phi"] = float(phi + e2)
            gates.append(g)
            busy[a] = busy[b] = True
            cur[a] = cur[b] = two_qubit
        for q in range(n):
            if busy[q]:
                continue
            if prev[q] in TWO_QUBIT_KINDS:
                k = "x12" if int(rng.integers(0, 2)) == 0 else "y12"
            elif prev[q] in ("x12", "y12", "h"):
                k = "t"
            else:
                k = ""
            if k:
                gates.append({"cycle": cyc, "kind": k, "qubits": [q]})
            cur[q] = k
        prev = cur
    gates += [{"cycle": depth + 1, "kind": "h", "qubits": [q]} for q in range(n)]
    return {"n_qubits": n, "xy": [list(p) for p in xy], "depth": depth, "gates": gates,
            "name": name}


def grid_rqc(rows: int, cols: int, depth: int, seed: int, **kw) -> dict:
    return rqc(grid_layout(rows, cols), depth, seed,
               name=kw.pop("name", "%dx%d_1+%d+1" % (rows, cols, depth)), **kw)


def diamond_rqc(depth: int, seed: int, **kw) -> dict:
    return rqc(diamond_layout(), depth, seed, name=kw.pop("name", "diamond70_1+%d+1" % depth),
               **kw)


def fsim_batch(n_circuits: int, depth: int = 12, sizes=(4, 5, 6), seed: int = 5000,
               jitter_seed0: int = 5900, theta: float = math.pi / 2, phi: float = math.pi / 6,
               jitter_sd: float = 0.02) -> list[dict]:
    """Circuits of uneven grid sizes with jittered fSim gates (rows, cols drawn from sizes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_circuits):
        r = int(sizes[int(rng.integers(0, len(sizes)))])
        c = int(sizes[int(rng.integers(0, len(sizes)))])
        out.append(grid_rqc(r, c, depth, seed + 1 + i, two_qubit="fsim", theta=theta, phi=phi,
                            jitter_sd=jitter_sd, jitter_seed=jitter_seed0 + i))
    return out


# ----------------------------------------------------------------------------- variants
def without_kinds(circ: dict, kinds) -> dict:
    """Copy of ``circ`` with every gate of the given kinds removed."""
    out = dict(circ)
    out["gates"] = [dict(g) for g in circ["gates"] if g["kind"] not in kinds]
    return out


def replace_two_qubit(circ: dict, kind: str, theta: float = 0.0, phi: float = 0.0) -> dict:
    """Copy of ``circ`` with every two-qubit gate replaced by ``kind`` (fsim angles given)."""
    out = dict(circ)
    gs = []
    for g in circ["gates"]:
        g = dict(g)
        if len(g["qubits"]) == 2:
            g["kind"] = kind
            g.pop("theta", None)
            g.pop("phi", None)
            if kind == "fsim":
                g["theta"], g["phi"] = float(theta), float(phi)
        gs.append(g)
    out["gates"] = gs
    return out


def fsim_params(circ: dict) -> np.ndarray:
    """[n_fsim, 2] array of (theta, phi) in gate-list order."""
    return np.array([[g["theta"], g["phi"]] for g in circ["gates"] if g["kind"] == "fsim"],
                    dtype=np.float64).reshape(-1, 2)


def with_fsim_params(circ: dict, params) -> dict:
    """Copy of ``circ`` with fSim angles replaced, in gate-list order."""
    params = np.asarray(params, dtype=np.float64).reshape(-1, 2)
    out = dict(circ)
    gs, i = [], 0
    for g in circ["gates"]:
        g = dict(g)
        if g["kind"] == "fsim":
            g["theta"], g["phi"] = float(params[i, 0]), float(params[i, 1])
            i += 1
        gs.append(g)
    if i != len(params):
        raise ValueError("expected %d fSim parameter pairs, got %d" % (i, len(params)))
    out["gates"] = gs
    return out


# ----------------------------------------------------------------------------- bit-strings
def bitstrings(n_qubits: int, m: int, seed: int, open_qubits=()) -> np.ndarray:
    """[m, n_qubits] uint8 uniform bits from PCG64(seed); open qubits are set to 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(0, 2, size=(m, n_qubits), dtype=np.uint8)
    if len(open_qubits):
        bits[:, list(open_qubits)] = 0
    return bits


def sampling_draws(n_batches: int, batch_len: int, n_c: int, seed: int):
    """Random numbers of the frugal sampler, as inputs: order [n_batches, n_c] int32, each row
    the first n_c entries of a uniformly random permutation of [0, batch_len) (a random subset
    without repetition, in random order), and u [n_batches, n_c] float64 uniform in [0, 1);
    both from PCG64(seed)."""
    if not 1 <= n_c <= batch_len:
        raise ValueError("need 1 <= n_c <= batch_len")
    rng = np.random.Generator(np.random.PCG64(seed))
    order = np.argsort(rng.random((n_batches, batch_len)), axis=1)[:, :n_c].astype(np.int32)
    u = rng.random((n_batches, n_c))
    return np.ascontiguousarray(order), u


def porter_thomas_amplitudes(n_batches: int, batch_len: int, n_qubits: int, seed: int):
    """[n_batches, batch_len] complex128 synthetic amplitudes with Porter-Thomas statistics:
    independent complex Gaussians of variance 1 / 2^n_qubits (so 2^n |a|^2 ~ Exp(1)), from
    PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sd = math.sqrt(0.5 / 2.0 ** n_qubits)
    z = rng.standard_normal((n_batches, batch_len, 2)) * sd
    return z[..., 0] + 1j * z[..., 1]


def grid_ids(rows_cols, cells) -> list[int]:
    """Row-major ids of (r, c) cells on a rows x cols grid."""
    _, cols = rows_cols
    return [r * cols + c for r, c in cells]


def dumps(circ: dict) -> str:
    return json.dumps(circ, sort_keys=True)


def loads(s: str) -> dict:
    return json.loads(s)
