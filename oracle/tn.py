"""E2: FP64 tensor-network contraction of an RQC with explicit slicing over cut bonds, plus
E3, its gradient by automatic differentiation.  TEST INFRASTRUCTURE (see
``oracle/__init__.py``).

Follows the paper's description step by step, in plain torch complex128 CPU ops:

* A circuit with fixed input |0..0> and output x is a tensor network (Methods B).
* Each two-qubit gate is split across its qubits along its Schmidt-style bond
  (Methods B: the bond dimension is the Schmidt rank, 2 for CZ and any diagonal gate, 4 for
  iSWAP).  Reading used: G = sum_k A_k (x) B_k in the elementary basis of q0, the
  lower-id qubit: if both off-diagonal 2x2 blocks of G are exactly zero,
  A_k = |k><k|, B_k = G_kk (k = 0, 1); otherwise k = 2i + j, A_k = |i><j|, B_k = G_ij, where
  G_ij[a, b] = <i a|G|j b>.
* Collapsing each qubit's gates along time gives one tensor per qubit,
  T_q[o, bonds] = <o| P_last ... P_1 |0>, with the output bit o left as an index and one
  bond index per neighbouring link (Methods B.1).  A link's bond is the mixed-radix index
  of the gates on that link, earliest gate most significant.
* A cut fixes the value of a bond; the amplitude is the sum over cut values ("paths") of the
  contraction with the cut bonds fixed (Methods B.1, cutting indexes).  The slice id is the
  mixed-radix index over the cuts in the order given, first cut most significant.
* Summing only a subset of paths gives the low-fidelity amplitudes of Methods C.1.

The contraction order only changes rounding, never the value (any order of pairwise
contractions of a tensor network gives the same result); ``order`` exists so that large
grids stay within memory.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gates as G

CDT = torch.complex128


def _tensor(m) -> torch.Tensor:
    return torch.as_tensor(np.asarray(m), dtype=CDT)


def fsim_t(theta: torch.Tensor, phi: torch.Tensor) -> torch.Tensor:
    c = torch.cos(theta).to(CDT)
    s = torch.sin(theta).to(CDT)
    one = torch.ones((), dtype=CDT)
    zero = torch.zeros((), dtype=CDT)
    e = torch.exp(-1j * phi.to(CDT))
    rows = [[one, zero, zero, zero],
            [zero, c, -1j * s, zero],
            [zero, -1j * s, c, zero],
            [zero, zero, zero, e]]
    return torch.stack([torch.stack(r) for r in rows])


def gate_tensor(g: dict, params=None, fsim_idx=None) -> torch.Tensor:
    if g["kind"] == "fsim" and params is not None:
        j = fsim_idx[id(g)]
        return fsim_t(params[j, 0], params[j, 1])
    return _tensor(G.matrix(g))


def split_two_qubit(mat4: torch.Tensor):
    """Bond decomposition of a 4x4 gate in the |lo hi> basis: list of (A_k, B_k)."""
    g = mat4.reshape(2, 2, 2, 2)  # [i, a, j, b] = <i a|G|j b>
    off_zero = bool(torch.all(g[0, :, 1, :] == 0)) and bool(torch.all(g[1, :, 0, :] == 0))
    pieces = []
    if off_zero:
        for k in range(2):
            a = torch.zeros(2, 2, dtype=CDT)
            a[k, k] = 1
            pieces.append((a, g[k, :, k, :]))
    else:
        for i in range(2):
            for j in range(2):
                a = torch.zeros(2, 2, dtype=CDT)
                a[i, j] = 1
                pieces.append((a, g[i, :, j, :]))
    return pieces


def _canonical(g: dict, mat: torch.Tensor):
    """(lo, hi, matrix in |lo hi> basis) for a two-qubit gate."""
    a, b = g["qubits"]
    if a < b:
        return a, b, mat
    sw = _tensor(G.SWAP)
    return b, a, sw @ mat @ sw


class Network:
    """Per-qubit tensors of a circuit after time collapse, with labelled indices."""

    def __init__(self, circ: dict, params: torch.Tensor | None = None):
        self.circ = circ
        self.n = circ["n_qubits"]
        gates = sorted(circ["gates"], key=lambda g: g["cycle"])
        fsim_idx = {}
        for g in circ["gates"]:
            if g["kind"] == "fsim":
                fsim_idx[id(g)] = len(fsim_idx)
        # links: (lo, hi) -> list of ranks of its gates in time order
        self.link_ranks: dict[tuple[int, int], list[int]] = {}
        # per qubit: list of (kind, payload) in time order
        timeline = [[] for _ in range(self.n)]
        for g in gates:
            mat = gate_tensor(g, params, fsim_idx)
            if len(g["qubits"]) == 1:
                timeline[g["qubits"][0]].append(("u", mat))
                continue
            lo, hi, m4 = _canonical(g, mat)
            pieces = split_two_qubit(m4)
            ranks = self.link_ranks.setdefault((lo, hi), [])
            gi = len(ranks)
            ranks.append(len(pieces))
            timeline[lo].append(("bond", ((lo, hi), gi, torch.stack([p[0] for p in pieces]))))
            timeline[hi].append(("bond", ((lo, hi), gi, torch.stack([p[1] for p in pieces]))))
        self.link_dim = {l: int(np.prod(r)) for l, r in self.link_ranks.items()}
        self.tensors = {}
        for q in range(self.n):
            self.tensors[q] = self._collapse(q, timeline[q])

    def _collapse(self, q, pieces):
        v = torch.zeros(2, dtype=CDT)
        v[0] = 1.0
        axes = []  # (link, gate index in link) of each bond axis of v, before the state axis
        for kind, p in pieces:
            if kind == "u":
                v = torch.einsum("ts,...s->...t", p, v)
            else:
                link, gi, mats = p
                v = torch.einsum("kts,...s->...kt", mats, v)
                axes.append((link, gi))
        # v[..., o] = <o| ... |0>; put o first
        v = torch.movedim(v, -1, 0)
        links = sorted({a[0] for a in axes}, key=lambda l: l[0] + l[1] - q)
        order = [0]
        shape = [2]
        labels = ["o%d" % q]
        for l in links:
            mine = sorted((gi, 1 + i) for i, (ll, gi) in enumerate(axes) if ll == l)
            order += [ax for _, ax in mine]
            shape.append(self.link_dim[l])
            labels.append("L%d_%d" % l)
        v = v.permute(order).reshape(shape)
        return v, labels

    # ------------------------------------------------------------------ contraction
    @staticmethod
    def _pair(a, b):
        (ta, la), (tb, lb) = a, b
        shared = [x for x in la if x in lb]
        ia = [la.index(x) for x in shared]
        ib = [lb.index(x) for x in shared]
        t = torch.tensordot(ta, tb, dims=(ia, ib))
        return t, [x for x in la if x not in shared] + [x for x in lb if x not in shared]

    @staticmethod
    def _size_after(a_labels, a_shape, b_labels, b_shape):
        da = dict(zip(a_labels, a_shape))
        db = dict(zip(b_labels, b_shape))
        s = 1
        for x, d in list(da.items()) + list(db.items()):
            if not (x in da and x in db):
                s *= d
        return s

    def _sweep(self, acc, items: dict):
        """Absorb every item into acc one at a time, smallest result first (ties: lowest id)."""
        items = dict(items)
        while items:
            if acc is None:
                q = min(items)
                acc = items.pop(q)
                continue
            best = None
            for q, it in sorted(items.items()):
                s = self._size_after(acc[1], acc[0].shape, it[1], it[0].shape)
                shared = any(x in acc[1] for x in it[1])
                key = (0 if shared else 1, s, q)
                if best is None or key < best[0]:
                    best = (key, q)
            acc = self._pair(acc, items.pop(best[1]))
        return acc

    def slice_tensors(self, x, open_qubits, cut_values: dict):
        """Qubit tensors with closed outputs fixed to x and cut bonds fixed."""
        out = {}
        for q in range(self.n):
            t, lab = self.tensors[q]
            if q not in open_qubits:
                t = t[int(x[q])]
                lab = lab[1:]
            for link, val in cut_values.items():
                name = "L%d_%d" % link
                if name in lab:
                    ax = lab.index(name)
                    t = t.select(ax, int(val))
                    lab = lab[:ax] + lab[ax + 1:]
            out[q] = (t, lab)
        return out

    def _in_order(self, acc, items: dict, qs):
        for q in qs:
            acc = items[q] if acc is None else self._pair(acc, items[q])
        return acc

    def contract(self, items: dict, order=None, open_qubits=()):
        """Contract labelled tensors; ``order`` is a list of ("region"|"sweep", qubits[,
        "fixed"]): a region is contracted on its own and then merged into the running result,
        a sweep absorbs its qubits into the running result one by one.  Qubits are taken
        smallest-result-first unless the segment is marked "fixed" (then in list order)."""
        if order is None:
            order = [("sweep", sorted(items))]
        acc = None
        for seg in order:
            kind, qs = seg[0], seg[1]
            fixed = len(seg) > 2 and seg[2] == "fixed"
            sub = {q: items[q] for q in qs}
            if kind == "region":
                r = self._in_order(None, sub, qs) if fixed else self._sweep(None, sub)
                acc = r if acc is None else self._pair(acc, r)
            else:
                acc = self._in_order(acc, sub, qs) if fixed else self._sweep(acc, sub)
        t, lab = acc
        want = ["o%d" % q for q in open_qubits]
        if sorted(lab) != sorted(want):
            raise RuntimeError("contraction left labels %r, expected %r" % (lab, want))
        if want:
            t = t.permute([lab.index(w) for w in want]).reshape(-1)
        return t

    def cut_dims(self, cuts):
        return [self.link_dim[tuple(sorted(c))] for c in cuts]

    def amplitudes(self, bits, open_qubits=(), cuts=(), slice_ids=None, order=None):
        """Sum over ``slice_ids`` (all slices if None) of the path amplitudes, [m, 2^n_open]
        (or [m] without open qubits).  With ``slice_ids=None`` the cut bonds are simply
        summed inside the contraction."""
        open_qubits = list(open_qubits)
        bits = np.asarray(bits)
        cuts = [tuple(sorted(c)) for c in cuts]
        dims = self.cut_dims(cuts)
        rows = []
        for x in bits:
            if slice_ids is None:
                rows.append(self.contract(self.slice_tensors(x, open_qubits, {}), order,
                                          open_qubits))
                continue
            acc = 0
            for s in slice_ids:
                vals, r = {}, int(s)
                for link, d in zip(reversed(cuts), reversed(dims)):
                    vals[link] = r % d
                    r //= d
                acc = acc + self.contract(self.slice_tensors(x, open_qubits, vals), order,
                                          open_qubits)
            rows.append(acc)
        out = torch.stack([torch.as_tensor(r, dtype=CDT).reshape(-1) for r in rows])
        return out if open_qubits else out[:, 0]


def quadrant_order(rows: int, cols: int):
    """A contraction order for a rows x cols grid split into quadrants A|B over C|D at
    (rows//2, cols//2), used only to bound memory (any order gives the same value): A row by
    row; B from its right edge inwards, its first column last; D bottom-up, each row right to
    left; finally C swept into the running result row by row, right to left."""
    rs, cs = rows // 2, cols // 2
    q = lambda r, c: r * cols + c  # noqa: E731
    A = [q(r, c) for r in range(rs) for c in range(cs)]
    B = [q(r, c) for r in range(rs) for c in range(cols - 1, cs, -1)] + \
        [q(r, cs) for r in range(rs)]
    D = [q(r, c) for r in range(rows - 1, rs - 1, -1) for c in range(cols - 1, cs - 1, -1)]
    C = [q(r, c) for r in range(rs, rows) for c in range(cs - 1, -1, -1)]
    return [("region", A, "fixed"), ("region", B, "fixed"), ("region", D, "fixed"),
            ("sweep", C, "fixed")]


def amplitudes(circ, bits, open_qubits=(), cuts=(), slice_ids=None, order=None):
    """numpy complex128 convenience wrapper around Network.amplitudes."""
    with torch.no_grad():
        return Network(circ).amplitudes(bits, open_qubits, cuts, slice_ids, order).numpy()


def num_slices(circ, cuts) -> int:
    net = Network(circ)
    return int(np.prod(net.cut_dims(cuts))) if cuts else 1


def linear_xeb_grad(circ, bits, order=None):
    """E3: linear XEB F = (2^n/m) sum |psi|^2 - 1 and dF/d(theta, phi) [n_fsim, 2] by
    torch autograd through the FP64 contraction."""
    params0 = np.array([[g["theta"], g["phi"]] for g in circ["gates"] if g["kind"] == "fsim"],
                       dtype=np.float64).reshape(-1, 2)
    params = torch.tensor(params0, requires_grad=True)
    net = Network(circ, params)
    psi = net.amplitudes(bits, order=order)
    n = circ["n_qubits"]
    f = (2.0 ** n) * torch.mean(psi.abs() ** 2) - 1.0
    f.backward()
    return float(f.detach()), params.grad.numpy().copy()


def amplitude_gate_grads(circ, bits, cot, open_qubits=(), cuts=(), slice_ids=None, order=None):
    """E3 for angles: with psi_i the amplitudes (the partial sum over ``slice_ids`` when
    given) and cot_i = dL/dRe(psi_i) + i dL/dIm(psi_i), return dL/d(theta, phi) [n_fsim, 2] =
    Re sum_i conj(cot_i) dpsi_i/d(theta, phi)."""
    params0 = np.array([[g["theta"], g["phi"]] for g in circ["gates"] if g["kind"] == "fsim"],
                       dtype=np.float64).reshape(-1, 2)
    params = torch.tensor(params0, requires_grad=True)
    psi = Network(circ, params).amplitudes(bits, open_qubits, cuts, slice_ids, order)
    c = torch.as_tensor(np.asarray(cot), dtype=CDT)
    # L = Re sum conj(cot) psi has dL/dRe psi + i dL/dIm psi = cot
    loss = torch.real(torch.sum(torch.conj(c) * psi))
    loss.backward()
    return params.grad.numpy().copy()
