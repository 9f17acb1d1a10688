"""Python binding of libqflex (names follow the C ABI; every step runs in the library).

    grid = build_grid(circuits, open_qubits=[...])
    amps = grid.contract_amplitudes(bits)            # torch complex128 on the GPU
"""
from __future__ import annotations

import ctypes as C
import json

import numpy as np

from . import _ffi as F


class _CircuitPack:
    """Keeps the ctypes arrays of circuits alive while the library reads them."""

    def __init__(self, circuits):
        self.keep = []
        arr = (F.Circuit * len(circuits))()
        for i, c in enumerate(circuits):
            n = int(c["n_qubits"])
            xy = (C.c_int32 * (2 * n))(*[int(v) for p in c["xy"] for v in p])
            gates = (F.Gate * max(1, len(c["gates"])))()
            for j, g in enumerate(c["gates"]):
                qs = list(g["qubits"])
                gates[j].cycle = int(g["cycle"])
                gates[j].kind = F.KIND[g["kind"]]
                gates[j].q0 = int(qs[0])
                gates[j].q1 = int(qs[1]) if len(qs) > 1 else -1
                gates[j].theta = float(g.get("theta", 0.0))
                gates[j].phi = float(g.get("phi", 0.0))
                if "mat" in g:
                    m = np.asarray(g["mat"], dtype=np.complex128).ravel()
                    buf = (C.c_double * (2 * m.size))(*np.stack([m.real, m.imag], 1).ravel())
                    self.keep.append(buf)
                    gates[j].mat = C.cast(buf, C.POINTER(C.c_double))
            self.keep += [xy, gates]
            arr[i].n_qubits = n
            arr[i].xy = C.cast(xy, C.POINTER(C.c_int32))
            arr[i].gates = C.cast(gates, C.POINTER(F.Gate))
            arr[i].n_gates = len(c["gates"])
        self.arr = arr


def _options(precision="c64", plan="auto", max_tensor_elems=0, open_qubits=(),
             bitstring_batch=0, slice_mode="random", graph=False, autotune=False, fused="auto"):
    o = F.Options()
    o.precision = F.PREC[precision]
    o.plan_kind = F.PLAN[plan]
    o.max_tensor_elems = int(max_tensor_elems or 0)
    op = (C.c_int32 * max(1, len(open_qubits)))(*[int(q) for q in open_qubits])
    o.open_qubits = C.cast(op, C.POINTER(C.c_int32))
    o.n_open = len(open_qubits)
    o.bitstring_batch = int(bitstring_batch)
    o.slice_mode = F.SLICES[slice_mode]
    o.graph = 1 if graph else 0
    o.autotune = 1 if autotune else 0
    o.fused = {"auto": 0, True: 1, "require": 1, False: -1, "never": -1}[fused]
    return o, op


def _pack_bits(circuits, bits):
    """Concatenated uint8 rows and their prefix offsets (bit-strings per circuit) for one
    bit-string array per circuit, each [m, n_qubits] of that circuit (one bit-string may be
    given as [n_qubits]).  The library reads circuit c's rows at its own width, so a
    mis-shaped array would shift every later circuit's rows: it is rejected here."""
    if isinstance(bits, np.ndarray) or (len(circuits) == 1 and not isinstance(bits, list)):
        bits = [bits]
    if len(bits) != len(circuits):
        raise ValueError("need one bit-string array per circuit (%d circuits, %d arrays)"
                         % (len(circuits), len(bits)))
    rows = []
    for i, (circ, b) in enumerate(zip(circuits, bits)):
        b = np.asarray(b, dtype=np.uint8)
        n = int(circ["n_qubits"])
        if b.size == 0:
            b = b.reshape(0, n)
        elif b.ndim == 1 and b.size == n:
            b = b.reshape(1, n)
        if b.ndim != 2 or b.shape[1] != n:
            raise ValueError("circuit %d: bit-strings must be [m, %d], got shape %s"
                             % (i, n, tuple(b.shape)))
        rows.append(np.ascontiguousarray(b))
    offs = np.zeros(len(rows) + 1, dtype=np.int64)
    for i, b in enumerate(rows):
        offs[i + 1] = offs[i] + b.shape[0]
    flat = np.concatenate([b.ravel() for b in rows]) if offs[-1] else np.zeros(1, np.uint8)
    return flat, offs


def _pack_slices(circuits, slice_ids):
    """Concatenated slice ids and their prefix offsets, one list per circuit (a single list
    for a one-circuit grid)."""
    if len(circuits) == 1 and (len(slice_ids) == 0 or np.isscalar(slice_ids[0])):
        slice_ids = [slice_ids]
    if len(slice_ids) != len(circuits):
        raise ValueError("need one slice list per circuit (%d circuits, %d lists)"
                         % (len(circuits), len(slice_ids)))
    so = np.zeros(len(slice_ids) + 1, dtype=np.int64)
    for i, sl in enumerate(slice_ids):
        so[i + 1] = so[i] + len(sl)
    si = np.concatenate([np.asarray(sl, dtype=np.int64).ravel() for sl in slice_ids]) \
        if so[-1] else np.zeros(1, np.int64)
    return si, so


def _check_device_array(t, shape, name):
    """A contiguous complex128 CUDA tensor of `shape` (the library writes or reads exactly
    that many elements at its address)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128:
        raise ValueError("%s must be a complex128 tensor" % name)
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous tensor of shape %s, got %s"
                         % (name, tuple(shape), tuple(t.shape)))
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(0)


def plan_describe(circuit: dict, **opts) -> dict:
    """qflex_plan_describe: validate and plan one circuit on the host, without a GPU."""
    L = F.lib()
    pack = _CircuitPack([circuit])
    o, keep = _options(**opts)
    need = C.c_int64(0)
    F.check(L.qflex_plan_describe(pack.arr, C.byref(o), None, 0, C.byref(need)))
    buf = C.create_string_buffer(int(need.value))
    F.check(L.qflex_plan_describe(pack.arr, C.byref(o), buf, need.value, C.byref(need)))
    return json.loads(buf.value.decode())


class Grid:
    """qflex_grid handle (device-resident time-collapsed tensors of a batch of circuits)."""

    def __init__(self, circuits, precision="c64", plan="auto", max_tensor_elems=0,
                 open_qubits=(), bitstring_batch=0, slice_mode="random", graph=False,
                 autotune=False, stream=None, fused="auto"):
        L = F.lib()
        if isinstance(circuits, dict):
            circuits = [circuits]
        self.circuits = list(circuits)
        self.n_open = len(open_qubits)
        self.open_qubits = list(open_qubits)
        pack = _CircuitPack(self.circuits)
        o, keep = _options(precision, plan, max_tensor_elems, open_qubits, bitstring_batch,
                           slice_mode, graph, autotune, fused)
        h = C.c_void_p()
        F.check(L.qflex_build_grid(pack.arr, len(self.circuits), C.byref(o), _stream(stream),
                                   C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            F.lib().qflex_grid_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_gates(self, circuit_dict: dict, circuit: int = 0, stream=None):
        """qflex_update_gates: new gates (same structure) for circuit `circuit`; its qubit
        tensors are collapsed again, the plan and tuned kernels are kept."""
        pack = _CircuitPack([circuit_dict])
        F.check(F.lib().qflex_update_gates(self._h, int(circuit), pack.arr, _stream(stream)))
        self.circuits[circuit] = circuit_dict

    def num_slices(self, circuit: int = 0) -> int:
        t = C.c_int64()
        F.check(F.lib().qflex_num_slices(self._h, circuit, C.byref(t)))
        return int(t.value)

    def plan_cuts(self, circuit: int = 0) -> list[tuple[int, int]]:
        buf = (C.c_int32 * 128)()
        n = C.c_int32()
        F.check(F.lib().qflex_plan_cuts(self._h, circuit, buf, 64, C.byref(n)))
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]

    def last_stats(self) -> dict:
        s = F.Stats()
        F.check(F.lib().qflex_last_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in F.Stats._fields_}

    def set_profiling(self, enable: bool = True):
        F.check(F.lib().qflex_set_profiling(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        buf = (F.KernelStat * 64)()
        n = C.c_int32()
        F.check(F.lib().qflex_profile_read(self._h, buf, 64, C.byref(n)))
        return {buf[i].name.decode(): {"launches": buf[i].launches, "ms": buf[i].ms,
                                       "flops": buf[i].flops, "bytes": buf[i].bytes}
                for i in range(min(n.value, 64))}

    def contract_amplitudes(self, bits, fidelity: float = 1.0, seed: int = 0, slice_ids=None,
                            device: bool = True, stream=None, out=None,
                            accumulate: bool = False):
        """Amplitudes [total bit-strings, 2^n_open] complex128 (a torch CUDA tensor when
        ``device``, else numpy).  ``bits``: one uint8 array [m_c, n_c] per circuit (or a
        single array for one circuit).  ``slice_ids``: optional list per circuit.
        ``accumulate``: add this call's slice sums into ``out`` (a device tensor) instead of
        overwriting it (QFLEX_OUT_ACCUMULATE)."""
        if accumulate and (out is None or not device):
            raise ValueError("accumulate needs a device output tensor `out`")
        L = F.lib()
        flat, offs = _pack_bits(self.circuits, bits)
        namp = 1 << self.n_open
        sid = soff = None
        if slice_ids is not None:
            si, so = _pack_slices(self.circuits, slice_ids)
            sid = si.ctypes.data_as(C.POINTER(C.c_int64))
            soff = so.ctypes.data_as(C.POINTER(C.c_int64))
        total = int(offs[-1])
        if out is not None and not device:
            raise ValueError("out is a device tensor: it needs device=True")
        if device:
            import torch
            if out is not None:
                _check_device_array(out, (total, namp), "out")
            res = out if out is not None else torch.empty((total, namp), dtype=torch.complex128,
                                                          device="cuda")
            ptr = C.c_void_p(res.data_ptr())
        else:
            res = np.empty((total, namp), dtype=np.complex128)
            ptr = C.c_void_p(res.ctypes.data)
        F.check(L.qflex_contract_amplitudes(
            self._h, flat.ctypes.data_as(C.POINTER(C.c_uint8)),
            offs.ctypes.data_as(C.POINTER(C.c_int64)), float(fidelity), C.c_uint64(int(seed)),
            sid, soff, ptr, (3 if accumulate else 1) if device else 0, _stream(stream)))
        return res


def _gate_grad_sizes(circ):
    return [4 if len(g["qubits"]) == 1 else 16 for g in circ["gates"]]


def _contract_grad(self, bits, cotangent=None, fidelity: float = 1.0, seed: int = 0,
                   slice_ids=None, stream=None):
    """qflex_contract_grad with host outputs: dict with ``amps`` [total, 2^n_open],
    ``grad_gates`` (per circuit, list of 2x2 / 4x4 arrays, dL/dRe G + i dL/dIm G),
    ``grad_params`` (per circuit [n_gates, 2]: dL/dtheta, dL/dphi), ``loss`` (per circuit
    linear XEB when no cotangent is given).  ``cotangent``: dL/dRe(amp) + i dL/dIm(amp) (what
    torch autograd passes for a complex tensor), numpy or torch (CPU or CUDA)."""
    L = F.lib()
    flat, offs = _pack_bits(self.circuits, bits)
    namp = 1 << self.n_open
    total = int(offs[-1])
    sid = soff = None
    keep = []
    if slice_ids is not None:
        si, so = _pack_slices(self.circuits, slice_ids)
        keep += [so, si]
        sid = si.ctypes.data_as(C.POINTER(C.c_int64))
        soff = so.ctypes.data_as(C.POINTER(C.c_int64))
    cot_ptr, cot_dev = None, 0
    if cotangent is not None:
        if hasattr(cotangent, "is_cuda") and cotangent.is_cuda:
            import torch
            cotangent = cotangent.to(torch.complex128).contiguous()
            if cotangent.numel() != total * namp:
                raise ValueError("cotangent must hold [%d, %d] values, got shape %s"
                                 % (total, namp, tuple(cotangent.shape)))
            keep.append(cotangent)
            cot_ptr, cot_dev = C.c_void_p(cotangent.data_ptr()), 1
        else:
            if hasattr(cotangent, "detach"):
                cotangent = cotangent.detach().cpu().numpy()
            c = np.ascontiguousarray(np.asarray(cotangent, dtype=np.complex128).reshape(total, namp))
            keep.append(c)
            cot_ptr = C.c_void_p(c.ctypes.data)
    amps = np.empty((total, namp), dtype=np.complex128)
    sizes = [_gate_grad_sizes(c) for c in self.circuits]
    n_entries = sum(sum(z) for z in sizes)
    n_gates = sum(len(z) for z in sizes)
    gg = np.empty(max(n_entries, 1), dtype=np.complex128)
    gp = np.empty((max(n_gates, 1), 2), dtype=np.float64)
    loss = np.empty(len(self.circuits), dtype=np.float64)
    F.check(L.qflex_contract_grad(
        self._h, flat.ctypes.data_as(C.POINTER(C.c_uint8)),
        offs.ctypes.data_as(C.POINTER(C.c_int64)), float(fidelity), C.c_uint64(int(seed)),
        sid, soff, cot_ptr, cot_dev, C.c_void_p(amps.ctypes.data), C.c_void_p(gg.ctypes.data),
        C.c_void_p(gp.ctypes.data), C.c_void_p(loss.ctypes.data), 0, _stream(stream)))
    out_gg, out_gp = [], []
    e0 = g0 = 0
    for z in sizes:
        lst = []
        for sz in z:
            d = 2 if sz == 4 else 4
            lst.append(gg[e0:e0 + sz].reshape(d, d).copy())
            e0 += sz
        out_gg.append(lst)
        out_gp.append(gp[g0:g0 + len(z)].copy())
        g0 += len(z)
    return {"amps": amps, "grad_gates": out_gg, "grad_params": out_gp, "loss": loss}


Grid.contract_grad = _contract_grad


def with_fsim_angles(circ: dict, params) -> dict:
    """Copy of a circuit with the angles of its fSim gates (in gate order) set from an
    [n_fsim, 2] array of (theta, phi)."""
    params = np.asarray(params, dtype=np.float64).reshape(-1, 2)
    out = dict(circ)
    gates, i = [], 0
    for g in circ["gates"]:
        g = dict(g)
        if g["kind"] == "fsim":
            g["theta"], g["phi"] = float(params[i, 0]), float(params[i, 1])
            i += 1
        gates.append(g)
    if i != len(params):
        raise ValueError("circuit has %d fSim gates, got %d angle pairs" % (i, len(params)))
    out["gates"] = gates
    return out


def _fsim_rows(circ):
    return [i for i, g in enumerate(circ["gates"]) if g["kind"] == "fsim"]


try:
    import torch

    class Amplitudes(torch.autograd.Function):
        """amplitudes = Amplitudes.apply(angles, circuit, bits, open_qubits, plan):
        complex128 amplitudes [m, 2^n_open] of ``circuit`` with its fSim angles replaced by
        ``angles`` ([n_fsim, 2] real tensor of (theta, phi)); differentiable in ``angles``
        through the adjoint contraction of libqflex."""

        # grids by circuit structure: a fitting loop changes only angles, so the plan and the
        # tensor layouts of its first call serve every later one (qflex_update_gates)
        _grids: dict = {}

        @staticmethod
        def _grid(circ, open_qubits, plan):
            key = (circ["n_qubits"], tuple(tuple(p) for p in circ["xy"]),
                   tuple((g["cycle"], g["kind"], tuple(g["qubits"])) for g in circ["gates"]),
                   tuple(open_qubits), plan)
            grid = Amplitudes._grids.get(key)
            if grid is not None:
                try:
                    grid.update_gates(circ)
                    return grid
                except F.QflexError:  # a rank change (e.g. theta = 0): build anew
                    Amplitudes._grids.pop(key, None)
            grid = Grid(circ, plan=plan, open_qubits=open_qubits)
            if len(Amplitudes._grids) >= 4:
                Amplitudes._grids.pop(next(iter(Amplitudes._grids)))
            Amplitudes._grids[key] = grid
            return grid

        @staticmethod
        def forward(ctx, angles, circuit, bits, open_qubits=(), plan="auto"):
            circ = with_fsim_angles(circuit, angles.detach().cpu().numpy())
            grid = Amplitudes._grid(circ, open_qubits, plan)
            ctx.grid, ctx.bits, ctx.rows = grid, np.asarray(bits, np.uint8), _fsim_rows(circ)
            ctx.circ = circ
            ctx.dtype, ctx.device = angles.dtype, angles.device
            amps = grid.contract_amplitudes(ctx.bits, device=torch.cuda.is_available())
            return amps.to(angles.device) if hasattr(amps, "to") else torch.from_numpy(amps)

        @staticmethod
        def backward(ctx, grad_amps):
            if ctx.grid.circuits[0] is not ctx.circ:  # a later forward updated the shared grid
                ctx.grid.update_gates(ctx.circ)
            res = ctx.grid.contract_grad(ctx.bits, cotangent=grad_amps)
            gp = torch.from_numpy(res["grad_params"][0][ctx.rows]).to(ctx.dtype).to(ctx.device)
            return gp, None, None, None, None
except ImportError:  # pragma: no cover
    pass


def select_slices(total: int, fidelity: float, seed: int, mode: str = "random") -> list:
    """qflex_select_slices: the ascending slice ids a contract call sums at this fidelity
    (host only)."""
    L = F.lib()
    ids = (C.c_int64 * max(1, int(total)))()
    n = C.c_int64(0)
    F.check(L.qflex_select_slices(int(total), float(fidelity), C.c_uint64(int(seed)),
                                  F.SLICES[mode], ids, int(total), C.byref(n)))
    return [int(ids[i]) for i in range(n.value)]


def build_grid(circuits, **kw) -> Grid:
    """qflex_build_grid."""
    return Grid(circuits, **kw)


def frugal_sample(amps, order, u, n_qubits: int, m: float = 10.0, stream=None, sync=True):
    """qflex_frugal_sample on device tensors: amps complex128 [n_batch, batch_len] (rows as
    Grid.contract_amplitudes returns them), order int32 [n_batch, n_c], u float64
    [n_batch, n_c].  Returns (accepted int32 [n_batch] on the device, -1 where a batch accepts
    nothing, and the error estimate as a float).  With sync=False the call only enqueues the
    kernels and returns the estimate as a one-element device tensor, without checking order
    for values outside the batch (accepted then holds -2 for such batches)."""
    import torch

    if amps.dim() != 2 or amps.dtype != torch.complex128 or not amps.is_cuda:
        raise ValueError("amps must be a complex128 CUDA tensor [n_batch, batch_len]")
    nb, blen = amps.shape
    if order.shape != u.shape or order.dim() != 2 or order.shape[0] != nb:
        raise ValueError("order and u must both be [n_batch, n_c]")
    if order.dtype != torch.int32 or u.dtype != torch.float64 or not (order.is_cuda and u.is_cuda):
        raise ValueError("order must be int32 and u float64, on the device")
    amps, order, u = amps.contiguous(), order.contiguous(), u.contiguous()
    accepted = torch.empty(nb, dtype=torch.int32, device=amps.device)
    partial = torch.empty(max(nb, 1), dtype=torch.float64, device=amps.device)
    tail = torch.zeros(1, dtype=torch.float64, device=amps.device)
    F.check(F.lib().qflex_frugal_sample(
        C.c_void_p(amps.data_ptr()), nb, blen, C.c_void_p(order.data_ptr()),
        C.c_void_p(u.data_ptr()), int(order.shape[1]), int(n_qubits), float(m),
        C.c_void_p(accepted.data_ptr()), C.c_void_p(partial.data_ptr()),
        C.c_void_p(tail.data_ptr()), _stream(stream)))
    if not sync:
        return accepted, tail
    if nb and bool((accepted == -2).any()):
        raise ValueError("order holds values outside [0, batch_len)")
    return accepted, float(tail.item()) if nb else 0.0


def fidelity_samples(grid: Grid, closed_bits, coins, uniform_bits, order, u, fidelity: float,
                     m: float = 10.0):
    """Fidelity-f samples (paper, Results, "Fraction of perfect fidelity amplitudes") by the
    frugal sampler: batch b (closed_bits[b], the open qubits' values ignored) gives an exact
    sample when coins[b] < f, else uniform_bits[b].  Only the exact batches are contracted, at
    full fidelity, and sampled on the device; the accepted open value is written into the open
    qubits, the first open qubit most significant (all in qflex_fidelity_samples).  One
    circuit per grid.  order / u: [n_batch, n_c] visit order and uniforms
    (rows of uniform batches are not used).  Returns (samples uint8 [n_batch, n], status int8
    [n_batch]: 1 exact sample, 0 uniform sample, -1 exact batch that accepted nothing)."""
    closed_bits = np.ascontiguousarray(closed_bits, dtype=np.uint8)
    uniform_bits = np.ascontiguousarray(uniform_bits, dtype=np.uint8)
    coins = np.ascontiguousarray(coins, dtype=np.float64)
    if closed_bits.ndim != 2 or closed_bits.shape[1] != int(grid.circuits[0]["n_qubits"]):
        raise ValueError("closed_bits must be [n_batch, %d]" % int(grid.circuits[0]["n_qubits"]))
    nb, n = closed_bits.shape
    if uniform_bits.shape != (nb, n) or coins.shape != (nb,):
        raise ValueError("closed_bits, uniform_bits [n_batch, n] and coins [n_batch] must agree")
    order = np.ascontiguousarray(order, dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.float64)
    if order.ndim != 2 or order.shape[0] != nb:
        raise ValueError("order and u must both be [n_batch, n_c]")
    if order.shape != u.shape:
        raise ValueError("order and u must both be [n_batch, n_c]")
    samples = np.empty((nb, n), dtype=np.uint8)
    status = np.empty(nb, dtype=np.int8)
    P = C.c_void_p
    F.check(F.lib().qflex_fidelity_samples(
        grid._h, P(closed_bits.ctypes.data), nb, P(coins.ctypes.data), float(fidelity),
        P(uniform_bits.ctypes.data), P(order.ctypes.data), P(u.ctypes.data), int(order.shape[1]),
        float(m), P(samples.ctypes.data), P(status.ctypes.data), _stream(None)))
    return samples, status