"""Host checks of the adjoint contraction's memory layout (the plan description's "grad" part):
the segments partition the steps, the checkpoints are exactly the intermediates that cross a
segment boundary, and a walk through the executor's schedule (forward over every step, then the
segments last to first, each but the last recomputed before it is reversed) never reads a value
or cotangent that a later write has overwritten.  Also: the layout takes less memory than
keeping every intermediate, and only it lets the 7x7 depth 1+40+1 (bond 32) gradient of one
bit-string fit one GPU."""
import pytest

import rqc_inputs as R
from paper_1811_09599_amd import plan_describe

OPEN_7x7 = [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)]
HBM_BYTES = 288e9


def _node(op):
    return int(op[1:]) if op.startswith("n") else None


class Memory:
    """Element ranges of the per-bit-string layout and what each one holds."""

    def __init__(self):
        self.held = []  # (start, end, tag)

    def write(self, start, size, tag):
        end = start + size
        self.held = [h for h in self.held if h[1] <= start or end <= h[0]]
        self.held.append((start, end, tag))

    def read(self, start, size, tag):
        assert (start, start + size, tag) in self.held, "%s overwritten or never written" % (tag,)


def _walk(plan, n_open):
    """Replay the executor's order of reads and writes on the layout."""
    g = plan["grad"]
    steps = plan["steps"]
    voff, coff, elems = g["voff"], g["coff"], g["node_elems"]
    mem = Memory()
    seg_of = {}
    for si, (a, b) in enumerate(g["segments"]):
        for k in range(a, b):
            seg_of[k] = si

    def val(v):
        return voff[v], elems[v], ("value", v)

    def cot(v):
        return coff[v], elems[v], ("cot", v)

    def forward(k):
        st = steps[k]
        for side, scratch in (("x", st["sx"]), ("y", st["sy"])):
            v = _node(st[side])
            if v is not None:
                mem.read(*val(v))
            if scratch >= 0:
                mem.write(*val(scratch))
        mem.write(*val(st["out"]))

    for k in range(len(steps)):
        forward(k)
    result = steps[-1]["out"]
    mem.read(*val(result))              # the amplitudes of a one-slice call
    mem.write(*cot(result))             # seed
    for si in range(len(g["segments"]) - 1, -1, -1):
        a, b = g["segments"][si]
        if si + 1 < len(g["segments"]):
            for k in range(a, b):
                forward(k)
        for k in range(b - 1, a - 1, -1):
            st = steps[k]
            mem.read(*cot(st["out"]))
            operands = []
            for side, scratch in (("x", st["sx"]), ("y", st["sy"])):
                v = _node(st[side])
                src = scratch if scratch >= 0 else v
                if src is not None:
                    mem.read(*val(src))
                operands.append(v)
            # the two operand cotangents land in the scratch rows, then are routed
            mem.write(g["s1off"], 1, ("s1", k))
            mem.write(g["s2off"], 1, ("s2", k))
            for v in operands:
                if v is not None:
                    mem.write(*cot(v))
    return g


CASES = [
    ("4x4 depth 16", lambda: R.grid_rqc(4, 4, 16, 1001), {}),
    ("5x4 depth 32 quadrant", lambda: R.grid_rqc(5, 4, 32, 1002), {"plan": "quadrant"}),
    ("6x6 fSim depth 12", lambda: R.fsim_batch(1, depth=12, sizes=(6,), seed=5000,
                                               jitter_seed0=5900)[0], {}),
    ("5x6 fSim depth 12", lambda: R.fsim_batch(1, depth=12, sizes=(5, 6), seed=5003,
                                               jitter_seed0=5903)[0], {}),
    ("7x7 depth 32 open batch", lambda: R.grid_rqc(7, 7, 32, 2000),
     {"open_qubits": "7x7"}),
    ("diamond 70 depth 24", lambda: R.diamond_rqc(24, 4001), {}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_gradient_layout_is_consistent(name, make, kw):
    circ = make()
    if kw.get("open_qubits") == "7x7":
        kw = dict(kw, open_qubits=R.grid_ids((7, 7), OPEN_7x7))
    plan = plan_describe(circ, **kw)
    steps = plan["steps"]
    g = plan["grad"]
    # segments: consecutive, in order, covering every step
    segs = g["segments"]
    assert segs[0][0] == 0 and segs[-1][1] == len(steps)
    assert all(segs[i][1] == segs[i + 1][0] and segs[i][0] < segs[i][1]
               for i in range(len(segs) - 1))
    seg_of = {k: si for si, (a, b) in enumerate(segs) for k in range(a, b)}
    # checkpoints: the intermediates produced in one segment and consumed in another
    producer = {st["out"]: k for k, st in enumerate(steps)}
    crossing = set()
    for k, st in enumerate(steps):
        for side in ("x", "y"):
            v = _node(st[side])
            if v is not None and seg_of[producer[v]] != seg_of[k]:
                crossing.add(v)
    assert set(g["checkpoints"]) == crossing
    assert g["elems"] == g["ckpt_elems"] + g["segment_elems"] + (g["s2off"] - g["s1off"]) + (
        g["elems"] - g["s2off"])
    assert g["elems"] <= g["store_all_elems"]
    # recomputation: every step at most once, the last segment never
    last = sum(st["flops"] for st in steps[segs[-1][0]:])
    assert g["recompute_flops"] == pytest.approx(sum(st["flops"] for st in steps) - last)
    _walk(plan, len(kw.get("open_qubits", ())))


def test_checkpoints_save_memory_where_it_matters():
    """A 6x6 fSim gradient keeps at most 1/3 of what storing every intermediate takes, and the
    7x7 depth 1+40+1 (bond 32) gradient of one bit-string fits the GPU's 288 GB only with
    checkpoints (a bond-32 intermediate is 2^30 complex64 elements, 8 GiB)."""
    c6 = R.fsim_batch(1, depth=12, sizes=(6,), seed=5000, jitter_seed0=5900)[0]
    g6 = plan_describe(c6)["grad"]
    assert 3 * g6["elems"] <= g6["store_all_elems"]
    c7 = R.grid_rqc(7, 7, 40, 3000)
    p7 = plan_describe(c7, open_qubits=R.grid_ids((7, 7), OPEN_7x7))
    g7 = p7["grad"]
    assert 8 * g7["store_all_elems"] > HBM_BYTES
    assert 8 * g7["elems"] < HBM_BYTES
    assert len(g7["segments"]) >= 2 and g7["checkpoints"]
