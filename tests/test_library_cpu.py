"""Host-side checks of libqflex: exported symbols, argument validation, planner, slice subset.
None of these launch GPU work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import rqc_inputs as R
from oracle import slices as OS
from paper_1811_09599_amd import _ffi as F
from paper_1811_09599_amd import plan_describe
from paper_1811_09599_amd.qflex import _CircuitPack, _options

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("qflex.h", "qflex_kernels.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(qflex_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = F.lib()
    declared = _declared()
    assert {"qflex_build_grid", "qflex_contract_amplitudes", "qflex_permute_c64",
            "qflex_gemm_c64"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(F.EXPORTS) == declared


def _status_describe(circ, **opts):
    L = F.lib()
    pack = _CircuitPack([circ])
    o, keep = _options(**opts)
    need = C.c_int64(0)
    st = L.qflex_plan_describe(pack.arr, C.byref(o), None, 0, C.byref(need))
    return st, L.qflex_last_error().decode()


def _status_build(circ, **opts):
    L = F.lib()
    pack = _CircuitPack([circ])
    o, keep = _options(**opts)
    h = C.c_void_p()
    st = L.qflex_build_grid(pack.arr, 1, C.byref(o), None, C.byref(h))
    assert not h.value or st == F.OK
    return st, L.qflex_last_error().decode()


def _bad_circuits():
    base = R.grid_rqc(3, 3, 8, 1)
    out = []
    c = dict(base, gates=[dict(g) for g in base["gates"]])
    c["gates"].append({"cycle": 3, "kind": "cz", "qubits": [0, 4]})  # diagonal pair
    out.append(("not unit distance", c))
    c = dict(base, gates=[dict(g) for g in base["gates"]])
    c["gates"].append({"cycle": 0, "kind": "t", "qubits": [2]})  # qubit 2 twice in cycle 0
    out.append(("used twice", c))
    c = dict(base, xy=[list(p) for p in base["xy"]])
    c["xy"][1] = list(c["xy"][0])
    out.append(("coordinates repeated", c))
    c = dict(base, gates=[dict(g) for g in base["gates"]])
    c["gates"].append({"cycle": 50, "kind": "h", "qubits": [9]})
    out.append(("out of range", c))
    return out


@pytest.mark.parametrize("why,circ", _bad_circuits())
def test_invalid_circuits_rejected_before_any_device_work(why, circ):
    for fn in (_status_describe, _status_build):
        st, msg = fn(circ)
        assert st == F.E_INVALID, (why, st, msg)
        assert msg


def test_invalid_options_rejected():
    c = R.grid_rqc(3, 3, 8, 1)
    assert _status_describe(c, open_qubits=list(range(9)) + [0])[0] == F.E_INVALID
    assert _status_describe(c, open_qubits=[12])[0] == F.E_INVALID
    assert _status_build(c, open_qubits=[3, 3])[0] == F.E_INVALID
    big = R.grid_rqc(5, 5, 8, 1)
    assert _status_describe(big, open_qubits=list(range(17)))[0] == F.E_INVALID


def test_invalid_mode_fields_rejected():
    """slice_mode and graph are checked with the other options, before any device work."""
    c = R.grid_rqc(3, 3, 8, 1)
    L = F.lib()
    pack = _CircuitPack([c])
    for field, bad in (("slice_mode", 2), ("slice_mode", -1), ("graph", 2), ("autotune", 3)):
        o, keep = _options()
        setattr(o, field, bad)
        h = C.c_void_p()
        assert L.qflex_build_grid(pack.arr, 1, C.byref(o), None, C.byref(h)) == F.E_INVALID, field
        assert not h.value


def test_plan_that_cannot_fit_is_reported():
    c = R.grid_rqc(4, 4, 16, 1)
    st, msg = _status_describe(c, plan="sweep", max_tensor_elems=64)
    assert st == F.E_PLAN and "max_tensor_elems" in msg
    st, msg = _status_build(c, plan="sweep", max_tensor_elems=64)
    assert st == F.E_PLAN


def test_build_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    st, msg = _status_build(R.grid_rqc(3, 3, 8, 1))
    assert st == F.E_DEVICE and msg


def test_planner_7x7_quadrant_matches_the_paper_structure():
    """SI A: two cuts on the 7x7 grid, four regions, every region tensor 2^(6 log2 D)."""
    for depth, d in ((32, 16), (40, 32)):
        c = R.grid_rqc(7, 7, depth, 2001)
        op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
        p = plan_describe(c, open_qubits=op)
        assert p["kind"] == "quadrant"
        assert [x[:2] for x in p["cuts"]] == [[20, 27], [44, 45]]
        assert [x[2] for x in p["cuts"]] == [int(np.log2(d))] * 2
        assert p["num_slices"] == d * d
        assert p["max_bits"] == 6 * int(np.log2(d))
        big = [s for s in p["steps"] if s["mb"] == s["kb"] == s["nb"] == 3 * int(np.log2(d))]
        assert len(big) == 2  # A.B and AB.D
        assert [s["deps"] for s in big] == [1, 3]


def test_plan_description_label_orders_are_consistent():
    """Each step lists its product's row, contracted and column labels and the storage orders
    of x and y: x holds exactly the rows and the contracted labels, y the contracted labels
    and the columns, and an intermediate x is the output of an earlier step with the rows and
    columns of that step."""
    op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    for c, kw in ((R.grid_rqc(7, 7, 32, 2000), {"open_qubits": op}),
                  (R.grid_rqc(5, 4, 16, 7), {"plan": "sweep"}),
                  (R.grid_rqc(4, 5, 16, 4242), {"plan": "cut_sweep", "max_tensor_elems": 1 << 8})):
        p = plan_describe(c, **kw)
        outs = {}
        for st in p["steps"]:
            assert sorted(st["x_in"]) == sorted(st["mlab"] + st["klab"])
            assert sorted(st["y_in"]) == sorted(st["klab"] + st["nlab"])
            assert len(st["mlab"]) == st["mb"] and len(st["klab"]) == st["kb"]
            assert len(st["nlab"]) == st["nb"]
            assert not set(st["mlab"]) & set(st["nlab"])
            for side in ("x", "y"):
                if st[side].startswith("n"):
                    lab = outs[int(st[side][1:])]
                    assert sorted(lab) == sorted(st[side + "_in"])
            outs[st["out"]] = st["mlab"] + st["nlab"]


@pytest.mark.parametrize("rows,cols,depth,seed,kw,n_open", [
    (7, 7, 32, 2000, {}, 6), (5, 4, 16, 7, {"plan": "sweep"}, 0),
    (4, 5, 16, 4242, {"plan": "cut_sweep", "max_tensor_elems": 1 << 8}, 2),
    (6, 6, 24, 3, {"plan": "quadrant"}, 3), (3, 5, 12, 11, {"plan": "auto"}, 1)])
def test_plan_contracts_every_tensor_once_and_counts_its_flops(rows, cols, depth, seed, kw,
                                                              n_open):
    """Whatever the plan kind: every qubit tensor and every intermediate is an operand of
    exactly one product, only the last product's output is left (holding just the open output
    labels), no tensor exceeds the plan's max_bits (nor the cap), and the plan's flops are the
    sum of its products' flops, each counted once per value of the cuts it depends on
    (slices are recomputed only from the first product that depends on their cut)."""
    c = R.grid_rqc(rows, cols, depth, seed)
    op = list(range(c["n_qubits"] - n_open, c["n_qubits"]))
    p = plan_describe(c, open_qubits=op, **kw)
    steps = p["steps"]
    uses = {}
    for st in steps:
        for side in ("x", "y"):
            uses[st[side]] = uses.get(st[side], 0) + 1
    assert set(uses.values()) == {1}
    assert sorted(int(k[1:]) for k in uses if k[0] == "q") == list(range(c["n_qubits"]))
    consumed = {int(k[1:]) for k in uses if k[0] == "n"}
    assert [st["out"] for st in steps if st["out"] not in consumed] == [steps[-1]["out"]]
    assert len(steps[-1]["mlab"]) + len(steps[-1]["nlab"]) == n_open
    for st in steps:
        assert max(st["mb"] + st["kb"], st["kb"] + st["nb"], st["mb"] + st["nb"]) <= p["max_bits"]
    if "max_tensor_elems" in kw:
        assert 2 ** p["max_bits"] <= kw["max_tensor_elems"]
    bits = [cut[2] for cut in p["cuts"]]
    assert p["num_slices"] == 2 ** sum(bits)
    total = 0
    for st in steps:
        mult = 1
        for ci, b in enumerate(bits):
            if st["deps"] >> ci & 1:
                mult *= 2 ** b
        total += st["flops"] * mult
        assert st["flops"] == 8 * 2 ** (st["mb"] + st["kb"] + st["nb"])
    assert total == pytest.approx(p["flops_all_slices"], rel=1e-12)


def test_planner_small_grid_is_a_single_sweep():
    p = plan_describe(R.grid_rqc(4, 4, 16, 1))
    assert p["kind"] == "sweep" and p["num_slices"] == 1 and p["max_bits"] <= 12
    q = plan_describe(R.grid_rqc(4, 4, 16, 1), plan="quadrant")
    assert q["kind"] == "quadrant" and q["num_slices"] == 16


def test_planner_reuse_lowers_flops():
    """Steps that do not depend on a cut are charged once per bit-string."""
    c = R.grid_rqc(7, 7, 32, 2001)
    p = plan_describe(c)
    per_slice = sum(s["flops"] for s in p["steps"])
    assert p["flops_all_slices"] < p["num_slices"] * per_slice / 1.2


@pytest.mark.parametrize("total,f,seed", [(1024, 1 / 64, 2700), (256, 1.0, 1), (96, 0.25, 7),
                                          (1, 1.0, 3), (4096, 1 / 256, 4700)])
def test_slice_subset_matches_oracle(total, f, seed):
    L = F.lib()
    k = int(round(total * f))
    ids = (C.c_int64 * k)()
    n = C.c_int64()
    F.check(L.qflex_select_slices(total, f, seed, 0, ids, k, C.byref(n)))
    assert n.value == k
    assert list(ids) == OS.select(total, f, seed)


def test_slice_subset_rejects_bad_fidelity():
    L = F.lib()
    n = C.c_int64()
    assert L.qflex_select_slices(10, 0.25, 1, 0, None, 0, C.byref(n)) == F.E_PLAN
    assert L.qflex_select_slices(10, 0.0, 1, 0, None, 0, C.byref(n)) == F.E_INVALID
    assert L.qflex_select_slices(10, 1.5, 1, 0, None, 0, C.byref(n)) == F.E_INVALID
    assert L.qflex_select_slices(10, 0.5, 1, 2, None, 0, C.byref(n)) == F.E_INVALID  # mode
    assert L.qflex_select_slices(12, 0.25, 1, 1, None, 0, C.byref(n)) == F.OK
    assert L.qflex_select_slices(12, 5 / 12, 1, 1, None, 0, C.byref(n)) == F.E_PLAN  # 5 !| 12


@pytest.mark.parametrize("total,f,seed", [(1024, 1 / 64, 2700), (256, 1.0, 1), (96, 0.25, 7),
                                          (4096, 1 / 256, 4700), (256, 1 / 16, 11)])
def test_block_slice_subset_matches_oracle(total, f, seed):
    """Block mode: k consecutive ids from a seeded multiple of k (both sides from SplitMix64)."""
    L = F.lib()
    k = int(round(total * f))
    ids = (C.c_int64 * k)()
    n = C.c_int64()
    F.check(L.qflex_select_slices(total, f, seed, 1, ids, k, C.byref(n)))
    assert n.value == k
    got = list(ids)
    assert got == OS.select_block(total, f, seed)
    assert got == list(range(got[0], got[0] + k)) and got[0] % k == 0


def test_gemm_variant_choice():
    L = F.lib()
    # the 256x128 and 128x128 tiles in the 3-multiplication form
    assert L.qflex_gemm_variant(4096, 4096, 4096) == 9  # 512 tiles of 256x128
    assert L.qflex_gemm_variant(4096, 2048, 16) == 9    # 256 tiles: one per compute unit
    assert L.qflex_gemm_variant(2048, 2048, 16) == 10   # 128: 128x128 tiles instead
    assert L.qflex_gemm_variant(4096, 4096 + 64, 16) == 1
    assert L.qflex_gemm_variant(64, 64, 16) == 1
    assert L.qflex_gemm_variant(64, 8, 256) == 0
    assert L.qflex_gemm_variant(1 << 20, 256, 8) == 5   # short K
    assert L.qflex_gemm_variant(1 << 16, 16, 256) == 8   # rows on MFMA (8 < N <= 16)
    assert L.qflex_gemm_variant(1 << 16, 8, 256) == 3    # rows on vector FMAs
    assert L.qflex_gemm_variant(1 << 16, 24, 256) == 3
    assert L.qflex_gemm_variant(1 << 16, 4, 16) == 3
    assert L.qflex_gemm_variant(1 << 14, 16, 256) == 0  # 64 row blocks: SIMT tiles instead
    assert L.qflex_gemm_variant(16, 256, 1 << 16) == 7  # reduction-shaped, on MFMA
    assert L.qflex_gemm_variant(32, 256, 1 << 16) == 4  # ... more than 16 rows: vector kernel
    assert L.qflex_gemm_variant(16, 32, 1 << 16) == 4   # ... N not a multiple of 64
    assert L.qflex_gemm_variant(1 << 16, 256, 4) == 5   # short K
    assert L.qflex_gemm_variant(1 << 16, 8, 8) == 3     # rows kernel, 8-deep k-tile
    assert L.qflex_gemm_variant(1 << 16, 32, 8) == 5    # K = 8 rows tile only up to N = 16


def test_split_gemm_argument_checks_run_before_any_launch():
    """Host-side validation of the kernel-level split product (no device memory is touched:
    the pointers are never dereferenced when a check fails)."""
    L = F.lib()
    fake = C.c_void_p(1 << 20)  # 16-byte aligned, never dereferenced
    ws = L.qflex_gemm_split_workspace(256, 128, 64, 1)
    assert ws >= 2 * 4 * (256 * 64 + 128 * 64)

    def call(M=256, N=128, K=64, prec=F.PREC["split_fp16"], ws_bytes=ws, A=fake):
        return L.qflex_gemm_split_c64(A, fake, fake, M, N, K, 0, 0, 1, prec, fake, ws_bytes, None)

    assert call(prec=F.PREC["c64"]) == F.E_INVALID
    assert call(prec=7) == F.E_INVALID
    assert call(ws_bytes=ws - 1) == F.E_INVALID
    assert call(M=96) == F.E_INVALID      # not a power of two
    assert call(K=8) == F.E_INVALID       # below the kernel's k-tile
    assert call(A=C.c_void_p((1 << 20) + 8)) == F.E_INVALID  # misaligned operand


def test_split_tile_entry_checks_the_tile_before_any_launch():
    """The split product with a caller's tile rejects tiles out of range or not fitting M, N on
    the host, like every other argument check (nothing is launched)."""
    L = F.lib()
    fake = C.c_void_p(1 << 20)
    ws = L.qflex_gemm_split_workspace(256, 256, 64, 1)

    def call(tile, M=256, N=256):
        return L.qflex_gemm_split_c64_tile(fake, fake, fake, M, N, 64, 0, 0, 1,
                                           F.PREC["split_bf16"], tile, fake, ws, None)

    for tile in (-2, 6, 100):
        assert call(tile) == F.E_INVALID
    assert b"tile" in L.qflex_last_error()
    assert call(0, M=128) == F.E_INVALID   # 256x128
    assert call(4, M=128) == F.E_INVALID   # 256x128, 3-multiplication form
    assert call(3, N=128) == F.E_INVALID   # 128x256
    assert call(5, N=128) == F.E_INVALID
    assert call(4, M=256, N=64) == F.E_INVALID


def test_noalloc_split_product_checks_run_before_any_launch():
    """The no-allocation split product checks its arguments as the workspace entry point does
    and rejects a product whose split operands exceed its fixed scratch (2048^3 needs 64 MiB +
    256 bytes), all on the host, before touching the device."""
    L = F.lib()
    fake = C.c_void_p(1 << 20)  # 16-byte aligned, never dereferenced

    def call(M=256, N=128, K=64, batch=1, prec=F.PREC["split_bf16"], A=fake):
        return L.qflex_gemm_split_c64_noalloc(A, fake, fake, M, N, K, 0, 0, batch, prec, None)

    assert L.qflex_gemm_split_workspace(2048, 2048, 2048, 1) > F.NOALLOC_SCRATCH_BYTES
    assert L.qflex_gemm_split_workspace(2048, 2048, 1024, 1) <= F.NOALLOC_SCRATCH_BYTES
    assert call(M=2048, N=2048, K=2048) == F.E_INVALID
    assert b"scratch" in L.qflex_last_error()
    assert call(M=1024, N=1024, K=1024, batch=5) == F.E_INVALID  # 80 MiB over the batch
    assert call(prec=F.PREC["c64"]) == F.E_INVALID
    assert call(M=96) == F.E_INVALID
    assert call(A=C.c_void_p((1 << 20) + 8)) == F.E_INVALID
    assert call(batch=0) == F.E_INVALID


def test_autotune_cache_file_round_trip(tmp_path):
    """The autotuner's table: loading a file merges its entries, saving writes them back line
    for line, a malformed file is rejected and leaves the table as it was."""
    L = F.lib()
    L.qflex_autotune_cache_clear()
    assert L.qflex_autotune_cache_size() == 0
    lines = ["gfx950_cu256|c64|4096x4096x4096|t00|b1|ws0 9",
             "gfx950_cu256|splitbf|65536x256x256|b8|g11|q01|c0 6",
             "gfx942_cu304|c64|256x16x65536|t10|b25|ws1 8"]
    src = tmp_path / "tune.txt"
    src.write_text("\n".join(lines) + "\n")
    n = C.c_int64(-1)
    F.check(L.qflex_autotune_cache_load(str(src).encode(), C.byref(n)))
    assert n.value == 3 and L.qflex_autotune_cache_size() == 3
    out = tmp_path / "out.txt"
    F.check(L.qflex_autotune_cache_save(str(out).encode()))
    assert sorted(out.read_text().splitlines()) == sorted(lines)
    for bad in ("key 3\nbroken\n", "key -1\n", "key 2 extra\n"):
        (tmp_path / "bad.txt").write_text(bad)
        assert L.qflex_autotune_cache_load(str(tmp_path / "bad.txt").encode(), None) == F.E_INVALID
        assert L.qflex_autotune_cache_size() == 3
    assert L.qflex_autotune_cache_load(str(tmp_path / "missing.txt").encode(), None) == F.E_INVALID
    assert L.qflex_autotune_cache_load(None, None) == F.E_INVALID
    L.qflex_autotune_cache_clear()
    assert L.qflex_autotune_cache_size() == 0


def test_split_k_workspace_only_for_reduction_shapes():
    """qflex_gemm_c64_workspace is non-zero only when a product has few output tiles and a long
    K (host-only arithmetic)."""
    L = F.lib()
    assert L.qflex_gemm_c64_workspace(16, 16, 1 << 16, 4) > 0
    assert L.qflex_gemm_c64_workspace(4096, 4096, 4096, 1) == 0   # enough tiles
    assert L.qflex_gemm_c64_workspace(16, 16, 256, 1) == 0        # K too short to split
    # the workspace holds chunks x batch x M x N complex64 values
    ws = L.qflex_gemm_c64_workspace(16, 16, 1 << 16, 4)
    assert ws % (8 * 4 * 16 * 16) == 0


def test_cut_sweep_plan_fits_the_70_qubit_diamond():
    """The diamond (no full rectangle, so no quadrant plan) is swept with cut links: every
    intermediate fits 2^30 elements and the slices number 2^(cut bits)."""
    c = R.diamond_rqc(24, 4001)
    d = plan_describe(c)
    assert d["kind"] == "cut_sweep"
    assert d["max_bits"] <= 30 and len(d["cuts"]) >= 1
    xy = c["xy"]
    for q0, q1, bits in d["cuts"]:
        assert abs(xy[q0][0] - xy[q1][0]) + abs(xy[q0][1] - xy[q1][1]) == 1
        assert bits == 3  # three CZ gates per link at depth 24, one bit each
    assert d["num_slices"] == 2 ** sum(b for _, _, b in d["cuts"])
    # without cuts the same sweep would need a 2^33-element frontier
    with pytest.raises(F.QflexError):
        plan_describe(c, plan="sweep")


def test_cut_sweep_cuts_until_the_cap():
    c = R.grid_rqc(4, 5, 16, 4242)
    for cap_bits in (8, 6):
        d = plan_describe(c, plan="cut_sweep", max_tensor_elems=1 << cap_bits)
        assert d["kind"] == "cut_sweep"
        assert d["max_bits"] <= cap_bits and d["cuts"]
    assert not plan_describe(c, plan="cut_sweep", max_tensor_elems=1 << 10)["cuts"]  # fits


def test_frugal_sample_rejects_bad_arguments_before_any_launch():
    L = F.lib()
    P = C.c_void_p
    one = P(16)  # never dereferenced: every call below fails its argument checks first
    cases = [
        (None, 4, 16, one, one, 2, 10, 10.0),   # NULL amps
        (one, -1, 16, one, one, 2, 10, 10.0),   # n_batch < 0
        (one, 4, 0, one, one, 2, 10, 10.0),     # batch_len < 1
        (one, 4, 16, one, one, -1, 10, 10.0),   # n_c < 0
        (one, 4, 16, None, one, 2, 10, 10.0),   # NULL order with visits
        (one, 4, 16, one, one, 2, 0, 10.0),     # n_qubits < 1
        (one, 4, 16, one, one, 2, 10, 0.0),     # M <= 0
        (one, 4, 16, one, one, 2, 10, float("nan")),
        (one, 4, 16, one, one, 2, 10, float("inf")),
    ]
    for a, nb, bl, o, u, nc, nq, m in cases:
        st = L.qflex_frugal_sample(a, nb, bl, o, u, nc, nq, m, one, one, one, None)
        assert st == F.E_INVALID, (nb, bl, nc, nq, m)


def test_workspace_sizes_are_64_bit():
    """Sizes above 2^31 bytes come back whole (the size queries return int64_t)."""
    L = F.lib()
    assert L.qflex_gemm_split_workspace(1 << 16, 1 << 16, 1 << 12, 1) == \
        256 + 2 * 4 * ((1 << 28) + (1 << 28))


def test_fsim_half_depth_plans_like_cz_full_depth():
    """A two-qubit fSim gate has a rank-4 bond decomposition (2 bond bits) where CZ has rank 2,
    so a 1+t/2+1 fSim circuit collapses to the bond dimensions of a 1+t+1 CZ circuit: on the
    7x7 grid both get the same quadrant plan, cuts, slices and flops."""
    op = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    cz = plan_describe(R.grid_rqc(7, 7, 32, 2001), open_qubits=op)
    fs = plan_describe(R.grid_rqc(7, 7, 16, 2002, two_qubit="fsim", jitter_sd=0.02,
                                  jitter_seed=3), open_qubits=op)
    for key in ("kind", "cuts", "num_slices", "max_bits", "flops_all_slices"):
        assert cz[key] == fs[key], key


def test_automatic_plan_is_the_cheapest_that_fits():
    """The automatic choice builds every plan kind that fits the memory cap and keeps the one
    with the lowest estimated time: a small grid sweeps without cuts, the 7x7 D=16 grid takes
    the quadrant plan, the diamond the only kind that fits it, and on the 6x6 depth-32 grid,
    where an uncut sweep fits but runs 2^20-element intermediates through every step, the
    quadrant plan with two cuts is estimated faster and chosen."""
    op7 = R.grid_ids((7, 7), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    cases = [(R.grid_rqc(4, 4, 16, 1), (), "sweep"),
             (R.grid_rqc(7, 7, 32, 2000), op7, "quadrant"),
             (R.diamond_rqc(24, 4001), (), "cut_sweep"),
             (R.grid_rqc(6, 6, 32, 77), (), "quadrant")]
    for c, op, want in cases:
        auto = plan_describe(c, open_qubits=op)
        assert auto["kind"] == want
        costs = {}
        for k in ("sweep", "quadrant", "cut_sweep"):
            try:
                costs[k] = plan_describe(c, open_qubits=op, plan=k)["cost_estimate_s"]
            except F.QflexError as e:
                assert e.status == F.E_PLAN
        assert auto["cost_estimate_s"] == min(costs.values()) == costs[want]
    # an uncut sweep fits the 6x6 depth-32 grid too: the choice was a matter of cost
    assert plan_describe(R.grid_rqc(6, 6, 32, 77), plan="sweep")["cuts"] == []


def test_gather_run_encoding_reproduces_the_bit_map():
    """The gathered products receive each bit-deposit map (storage position of every index bit)
    as at most 8 runs of consecutive bits, packed s | len << 8 | d << 16 by the host.  For
    random maps, depositing an index through the runs equals depositing it bit by bit, and a map
    of more than 8 maximal runs is reported as 9 (the kernels then walk the bits)."""
    fn = getattr(F.lib(), "_ZN5qflex3dev11gather_runsEPKaiiPi")
    fn.restype = C.c_int32
    fn.argtypes = [C.POINTER(C.c_int8), C.c_int, C.c_int, C.POINTER(C.c_int32)]
    rng = np.random.default_rng(5)
    seen_overflow = seen_fit = 0
    for trial in range(400):
        n = int(rng.integers(3, 38))
        first = int(rng.integers(0, 3))
        if trial % 2:  # a few contiguous blocks of storage positions
            cuts = sorted(set(rng.integers(1, n, size=int(rng.integers(0, 6))).tolist()))
            blocks = np.split(np.arange(n), cuts)
            posl = []
            order = rng.permutation(len(blocks))  # the blocks land in storage in this order
            offs = np.cumsum([0] + [len(blocks[o]) for o in order])
            place = {int(o): int(offs[i]) for i, o in enumerate(order)}
            for bi, blk in enumerate(blocks):
                posl += [place[bi] + j for j in range(len(blk))]
        else:  # arbitrary distinct positions
            posl = rng.permutation(40)[:n].tolist()
        pos = (C.c_int8 * 40)(*(posl + [0] * (40 - n)))
        runs = (C.c_int32 * 8)()
        nr = fn(pos, first, n, runs)
        maximal = sum(1 for i in range(first, n) if i == first or posl[i] != posl[i - 1] + 1)
        if maximal > 8:
            assert nr == 9
            seen_overflow += 1
            continue
        assert nr == maximal
        seen_fit += 1
        for v in rng.integers(0, 2 ** (n - first), size=20).tolist():
            want = sum(((v >> (i - first)) & 1) << posl[i] for i in range(first, n))
            got = 0
            for r in range(nr):
                w = runs[r]
                s, ln, d = w & 0xFF, (w >> 8) & 0xFF, (w >> 16) & 0xFF
                got |= ((v >> s) & ((1 << ln) - 1)) << d
            assert got == want
    assert seen_overflow > 20 and seen_fit > 100

def test_fused_option_checked_before_any_device_work():
    """qflex_options.fused must be -1, 0 or 1, and 1 needs complex64: both are rejected by the
    option check, before the grid touches a device."""
    from paper_1811_09599_amd import qflex as Q
    L = F.lib()
    c = R.grid_rqc(2, 2, 4, 3)
    pack = Q._CircuitPack([c])
    for prec, fused in (("split_bf16", "require"), ("split_fp16", "require")):
        o, keep = Q._options(precision=prec, fused=fused)
        h = C.c_void_p()
        assert L.qflex_build_grid(pack.arr, 1, C.byref(o), None, C.byref(h)) == F.E_INVALID
        assert b"complex64" in L.qflex_last_error()
    o, keep = Q._options()
    o.fused = 2
    h = C.c_void_p()
    assert L.qflex_build_grid(pack.arr, 1, C.byref(o), None, C.byref(h)) == F.E_INVALID
    assert b"fused" in L.qflex_last_error()


def test_plan_describe_reports_the_fused_fit():
    """The fused small-plan kernel holds one bit-string's tensors in LDS: the arena, the free
    part of every qubit tensor, 32-byte step descriptors and 16-bit index tables (per step,
    2^mb + 2^nb + 2 * 2^kb entries), at most 144 KiB.  plan_describe reports the fit with these
    figures, recomputed here from the plan's own description; larger plans report why not."""
    cases = [((4, 4, 16, 1), {}), ((4, 4, 16, 1), {"open_qubits": [0, 5]}),
             ((4, 4, 16, 1), {"plan": "quadrant"}), ((3, 4, 24, 1), {"plan": "quadrant"}),
             ((6, 5, 16, 1), {}), ((4, 4, 16, 1), {"plan": "cut_sweep", "max_tensor_elems": 128})]
    for args, kw in cases:
        p = plan_describe(R.grid_rqc(*args), **kw)
        f = p["fused"]
        assert f["fits"] == 1, (args, kw, f)
        tab = sum(2 ** s["mb"] + 2 ** s["nb"] + 2 * 2 ** s["kb"] for s in p["steps"])
        image = p["arena_elems"] + sum(2 ** b for b in p["qubit_free_bits"])
        assert f["steps"] == len(p["steps"]) and f["table_entries"] == tab
        assert f["lds_bytes"] == 8 * image + 32 * len(p["steps"]) + 2 * tab
        assert f["lds_bytes"] <= 144 * 1024
    for args in ((6, 6, 16, 1), (7, 7, 40, 1)):
        f = plan_describe(R.grid_rqc(*args))["fused"]
        assert f["fits"] == 0 and "LDS" in f["why"], (args, f)


def test_python_marshalling_rejects_misshaped_inputs():
    """The library reads each circuit's bit-string rows at that circuit's width and writes or
    reads exactly [total, 2^n_open] values at an output or cotangent address, so the binding
    checks shapes before any call: one array per circuit, rows of n_qubits (one bit-string may
    be a 1-D row), empty arrays allowed, one slice list per circuit, a complex128 contiguous
    output of the exact shape."""
    import torch

    from paper_1811_09599_amd.qflex import _check_device_array, _pack_bits, _pack_slices
    cs = [R.grid_rqc(2, 2, 4, 1), R.grid_rqc(2, 3, 4, 2)]
    a, b = R.bitstrings(4, 3, 1), R.bitstrings(6, 2, 2)
    flat, offs = _pack_bits(cs, [a, b])
    assert list(offs) == [0, 3, 5] and flat.size == 3 * 4 + 2 * 6
    assert np.array_equal(flat[12:], b.ravel())  # circuit 1's rows after circuit 0's, at width 6
    flat, offs = _pack_bits(cs, [a[0], np.zeros((0,), np.uint8)])  # a 1-D row; an empty array
    assert list(offs) == [0, 1, 1] and flat.size == 4
    for bad in ([a], [a, a], [b, b], [a, b[:, :5]], [a.ravel(), b]):
        with pytest.raises(ValueError):
            _pack_bits(cs, bad)
    si, so = _pack_slices(cs, [[3, 1], []])
    assert list(so) == [0, 2, 2] and list(si[:2]) == [3, 1]
    with pytest.raises(ValueError):
        _pack_slices(cs, [[0]])
    si, so = _pack_slices(cs[:1], [2, 0])  # one circuit: a single list
    assert list(so) == [0, 2]
    for t in (torch.zeros((5, 2), dtype=torch.complex64), torch.zeros((5, 1), dtype=torch.complex128),
              torch.zeros((2, 5), dtype=torch.complex128).t()):
        with pytest.raises(ValueError, match="complex128|shape"):
            _check_device_array(t, (5, 2), "out")
    with pytest.raises(ValueError, match="CUDA"):  # right shape and type, host memory
        _check_device_array(torch.zeros((5, 2), dtype=torch.complex128), (5, 2), "out")
