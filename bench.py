"""Throughput of the RQC amplitude contraction on one MI355X.

Workload: 7x7 grid, depth 1+32+1 (bond dimension 16 on every link), the quadrant plan with
2 cut bonds (256 slices, all summed: fidelity 1), a 6-qubit open batch (64 amplitudes per
bit-string).  One step = one contraction call over the next `--bitstrings` bit-strings of a
seeded set of 1024, every slice included.  Three precisions are measured: split-bf16 (the
headline `value`), split-fp16 and complex64 (reported alongside), each with its error against
the FP64 oracle on sampled slices.

Prints one JSON line: amplitudes/s (whole job), sustained TFLOP/s of the plan (8 real flops
per complex multiply-add), the roofline of the dominant kernel measured with HIP events around
its launches in the timed region, and the CPU oracle timed on a bounded sample (the only part
that runs the oracle, together with the gradient's parity check).  Further workloads, each
under its own key: "fsim_7x7" (the headline workload with fSim couplers at depth 1+16+1),
"sampling" (frugal rejection sampling of one bit-string per open batch),
"gradient" (the adjoint contraction: 96 jittered-fSim circuits on 4x4 to 6x6 grids, depth
1+12+1, linear XEB over 128 bit-strings each, amplitudes and gradients of every fSim angle in
one call) and "diamond" (the 70-qubit diamond at fidelity 1/8); "ceilings" holds the vendor
GEMM and device copy rates of the same device.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--bitstrings 8]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: dense MFMA fp32 / bf16, fp32 vector without packed math, HBM3E
PEAK = {"mfma_fp32": (157.3, "TFLOP/s"), "mfma_bf16": (2500.0, "TFLOP/s"),
        "mfma_fp16": (2500.0, "TFLOP/s"),
        "alu": (78.6, "TFLOP/s"), "hbm": (8000.0, "GB/s")}
C64_TOL = 1e-5
# stated bounds of the 2^(n/2)-scaled amplitude error (max over the batch)
TOL = {"split_bf16": 2e-4, "split_fp16": 4 * C64_TOL, "c64": C64_TOL}
DTYPE = {"split_bf16": "bf16x3", "split_fp16": "fp16x3", "c64": "c64"}


def flop_peak(name):
    """The arithmetic peak a kernel's flops are measured against, from its name."""
    if name.startswith("gemm_split_bf16"):
        return "mfma", PEAK["mfma_bf16"][0]
    if name.startswith("gemm_split_fp16"):
        return "mfma", PEAK["mfma_fp16"][0]
    if name.startswith("gemm_mfma"):
        return "mfma", PEAK["mfma_fp32"][0]
    if name.startswith("gemm_"):  # SIMT, rows, reduce and short-K products: FP32 vector ALU
        return "alu", PEAK["alu"][0]
    return None, None


def roofline(prof):
    """Roofline of the kernel with the most time: its algorithmic flops and bytes per launch
    (recorded by the library with each launch) over its average launch time; the bound is the
    resource the kernel uses the larger fraction of."""
    name = max(prof, key=lambda k: prof[k]["ms"])
    k = prof[name]
    sec = k["ms"] * 1e-3
    gbps = k["bytes"] / sec / 1e9
    hbm_frac = gbps / PEAK["hbm"][0]
    kind, fpeak = flop_peak(name)
    tflops = k["flops"] / sec / 1e12
    flop_frac = tflops / fpeak if fpeak else 0.0
    if kind is None or hbm_frac >= flop_frac:
        bound, achieved, peak, unit = "hbm", gbps, PEAK["hbm"][0], "GB/s"
    else:
        bound, achieved, peak, unit = kind, tflops, fpeak, "TFLOP/s"
    return name, {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                  "frac": round(achieved / peak, 4), "traffic": None,
                  "flop_frac": round(flop_frac, 4), "hbm_frac": round(hbm_frac, 4),
                  "avg_launch_us": round(1e3 * k["ms"] / max(k["launches"], 1), 3),
                  "launches": k["launches"]}


def ceilings():
    """What this device sustains outside the library, measured in the same process: the vendor
    GEMM (torch.matmul, hipBLASLt) on 8192^3 random bf16 and fp32 operands, and a 1 GiB device
    to device copy (read + write bytes).  Context for the roofline fractions above."""
    import torch

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    out = {}
    n = 8192
    for dt, key in ((torch.bfloat16, "vendor_gemm_bf16_tflops"),
                    (torch.float32, "vendor_gemm_fp32_tflops")):
        a = torch.randn(n, n, dtype=dt, device="cuda")
        b = torch.randn(n, n, dtype=dt, device="cuda")
        c = torch.empty(n, n, dtype=dt, device="cuda")
        out[key] = round(2.0 * n ** 3 / timed(lambda: torch.matmul(a, b, out=c), 20) / 1e12, 1)
        del a, b, c
    src = torch.randn(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out["device_copy_gbps"] = round(2.0 * 4 * src.numel() / timed(lambda: dst.copy_(src), 10)
                                    / 1e9, 1)
    del src, dst
    # the library's split-bf16 product (qflex_gemm_split_c64 with A given transposed, so that
    # both operands are split by a pass of their own and the product kernel is the pre-split
    # one the headline's square steps run; the passes are included) on the 7x7 workload's
    # square shape, on random and then on constant operands: the same launches, differing only
    # in how many bits the data toggles
    import ctypes as C

    from paper_1811_09599_amd import _ffi as F
    L = F.lib()
    m, b = 4096, 4
    a = torch.randn(b, m, m, dtype=torch.complex64, device="cuda")
    bb = torch.randn(b, m, m, dtype=torch.complex64, device="cuda")
    c = torch.empty_like(a)
    nws = L.qflex_gemm_split_workspace(m, m, m, b)
    ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
    strm = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def split_product():
        F.check(L.qflex_gemm_split_c64(C.c_void_p(a.data_ptr()), C.c_void_p(bb.data_ptr()),
                                       C.c_void_p(c.data_ptr()), m, m, m, 1, 0, b,
                                       F.PREC["split_bf16"], C.c_void_p(ws.data_ptr()), nws,
                                       strm))

    flops = 24.0 * m ** 3 * b  # 3 real products per complex product on 16-bit MFMA
    out["split_bf16_4096cube_x4_random_tflops"] = round(flops / timed(split_product, 5) / 1e12, 1)
    a.fill_(complex(0.75, -0.5))
    bb.fill_(complex(0.25, 0.5))
    out["split_bf16_4096cube_x4_constant_tflops"] = round(flops / timed(split_product, 5) / 1e12,
                                                          1)
    del a, bb, c, ws
    out["note"] = ("hipBLASLt via torch.matmul at 8192^3 on random operands, a 1 GiB device "
                   "copy, and this library's split-bf16 product on random vs constant "
                   "operands, timed in this run: practical ceilings of this device next to the "
                   "published peaks (the product's MFMA rate depends on the data's power draw)")
    return out


def run_precision(precision, circ, open_q, all_bits, args):
    import torch

    from paper_1811_09599_amd import build_grid

    t0 = time.time()
    grid = build_grid(circ, open_qubits=open_q, precision=precision,
                      autotune=not args.no_autotune)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    B = args.bitstrings
    out = torch.empty((B, 64), dtype=torch.complex128, device="cuda")

    def step(i):
        lo = (i * B) % len(all_bits)
        grid.contract_amplitudes(all_bits[lo:lo + B], out=out)
        return grid.last_stats()["flops"]

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    grid.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flops = 0.0
    for i in range(args.steps):
        flops += step(args.warmup + i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = grid.profile_read()
    grid.set_profiling(False)
    dom, roof = roofline(prof)
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "avg_us": round(1e3 * v["ms"] / max(v["launches"], 1), 3),
                   "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                   "gbps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    amps = args.steps * B * 64
    return grid, {"value": amps / dt, "ms_per_step": 1e3 * dt / args.steps,
                  "tflops": flops / dt / 1e12, "dominant_kernel": dom, "roofline": roof,
                  "kernels": kernels, "grid_build_s": build_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--bitstrings", type=int, default=8, help="bit-strings per step")
    ap.add_argument("--precision", default="all",
                    choices=["all", "c64", "split_bf16", "split_fp16"])
    ap.add_argument("--cpu-slices", type=int, default=3, help="oracle sample size (slices)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gradient", action="store_true", help="skip the gradient workload")
    ap.add_argument("--no-diamond", action="store_true", help="skip the diamond workload")
    ap.add_argument("--no-sampling", action="store_true", help="skip the sampler workload")
    ap.add_argument("--no-fsim", action="store_true", help="skip the 7x7 fSim workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="kernel choice by shape rules only (default: the library's autotuner "
                         "times the variants of every step during the warm-up call)")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip timing the vendor GEMM and a device copy for context")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device to device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import rqc_inputs as R
    from paper_1811_09599_amd import plan_describe

    torch.cuda.set_device(0)
    if args.copy_probe:
        # a plain copy of known size: reads 1 GiB and writes 1 GiB; under rocprofv3 --pmc its
        # FETCH_SIZE / WRITE_SIZE give the scale of those counters on this device
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # measured first, on a device that has not been running the workloads yet
    ceil = None if args.no_ceilings else ceilings()
    rows = cols = 7
    circ = R.grid_rqc(rows, cols, 32, 2000)
    open_q = R.grid_ids((rows, cols), [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)])
    all_bits = R.bitstrings(rows * cols, 1024, 2500, open_q)
    plan = plan_describe(circ, open_qubits=open_q)
    precs = ["split_bf16", "split_fp16", "c64"] if args.precision == "all" else [args.precision]
    results, grids = {}, {}
    for p in precs:
        grids[p], results[p] = run_precision(p, circ, open_q, all_bits, args)
    head = precs[0]
    r = results[head]
    res = {
        "metric": "amplitudes/s", "value": r["value"], "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[head], "data": "synthetic",
        "config": {"workload": "7x7 RQC depth 1+32+1 (bond dim 16), quadrant plan with 2 cuts "
                               "(256 slices, fidelity 1), 6-qubit open batch (64 amplitudes "
                               "per bit-string), %d bit-strings per step" % args.bitstrings,
                   "grid": "7x7", "depth": "1+32+1", "slices": plan["num_slices"],
                   "fidelity": 1.0, "amplitudes_per_bitstring": 64,
                   "bitstrings_per_step": args.bitstrings,
                   "plan_flops_per_bitstring": plan["flops_all_slices"], "precision": head},
        "tflops": r["tflops"], "tflops_frac_fp32_mfma_peak": r["tflops"] / PEAK["mfma_fp32"][0],
        "dominant_kernel": r["dominant_kernel"], "roofline": r["roofline"],
        "kernels": r["kernels"], "grid_build_s": r["grid_build_s"],
        "precisions": {p: {k: v for k, v in results[p].items() if k != "kernels"}
                       for p in precs},
    }
    for p in precs:
        if p != "c64" and "c64" in results:
            res["speedup_%s_vs_c64" % p] = results[p]["value"] / results["c64"]["value"]
    if not args.no_fsim:
        # fSim couplers at half the depth: the same bond dimensions, plan and flops (1+t/2+1)
        circ_f = R.grid_rqc(rows, cols, 16, 2002, two_qubit="fsim", jitter_sd=0.02,
                            jitter_seed=3)
        g_f, r_f = run_precision(head, circ_f, open_q, all_bits, args)
        g_f.close()
        res["fsim_7x7"] = {
            "workload": "7x7 RQC with fSim(pi/2 + N(0, 0.02), pi/6 + N(0, 0.02)) couplers, depth "
                        "1+16+1 (bond dim 16, the CZ 1+32+1 plan), %s, other settings as the "
                        "headline" % head,
            "metric": "amplitudes/s", "unit": "amplitudes/s",
            **{k: r_f[k] for k in ("value", "ms_per_step", "tflops", "dominant_kernel",
                                   "roofline")}}
    if not args.no_sampling:
        res["sampling"] = run_sampling(grids[head].contract_amplitudes(all_bits[:4]),
                                       r["value"])
    grad_check = None
    if not args.no_gradient:
        res["gradient"], grad_check = run_gradient(args)
    if not args.no_diamond:
        res["diamond"] = run_diamond(args)
    if ceil:
        res["ceilings"] = ceil
    if not args.no_cpu_baseline:
        res.update(cpu_baseline(circ, grids, all_bits[:1], open_q, args.cpu_slices, rows, cols))
        if grad_check is not None:
            res["gradient"]["parity"] = gradient_parity(*grad_check)
    print(json.dumps(res), flush=True)


def run_diamond(args):
    """70-qubit diamond lattice, depth 1+24+1 (bond 8), cut sweep with 2^30-element
    intermediates, one amplitude per bit-string at fidelity 1/8 (one of the 8 slices, seeded),
    split-bf16 products; checked against complex64 on the same call."""
    import numpy as np
    import torch

    import rqc_inputs as R
    from paper_1811_09599_amd import build_grid

    circ = R.diamond_rqc(24, 4001)
    bits = R.bitstrings(70, 64, 4500)
    B = 4  # bit-strings per step
    t0 = time.time()
    grid = build_grid(circ, precision="split_bf16", autotune=not args.no_autotune)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    S = grid.num_slices()
    fid = 1.0 / S
    for i in range(max(args.warmup, 0)):
        grid.contract_amplitudes(bits[:B], fidelity=fid, seed=4700)
    torch.cuda.synchronize()
    grid.set_profiling(True)
    t0 = time.perf_counter()
    flops = 0.0
    steps = max(1, args.steps)
    for i in range(steps):
        lo = (i * B) % len(bits)
        grid.contract_amplitudes(bits[lo:lo + B], fidelity=fid, seed=4700)
        flops += grid.last_stats()["flops"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = grid.profile_read()
    grid.set_profiling(False)
    dom, roof = roofline(prof)
    top = sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:5]
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                   "gbps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in top}
    a = grid.contract_amplitudes(bits[:B], fidelity=fid, seed=4700).cpu().numpy()
    grid.close()
    ref = build_grid(circ).contract_amplitudes(bits[:B], fidelity=fid, seed=4700).cpu().numpy()
    err = scaled_errors(a, ref)
    return {"workload": "70-qubit diamond lattice, depth 1+24+1 (bond 8), cut sweep (%d cut "
                        "link, %d slices), fidelity 1/%d, one amplitude per bit-string, %d "
                        "bit-strings per step, split-bf16" % (len(grid_cuts(circ)), S, S, B),
            "metric": "amplitudes/s", "value": B * steps / dt, "unit": "amplitudes/s",
            "steps": steps, "ms_per_step": 1e3 * dt / steps, "tflops": flops / dt / 1e12,
            "dominant_kernel": dom, "roofline": roof, "kernels": kernels,
            "grid_build_s": build_s,
            "split_bf16_vs_c64": {"max_rel_err": err["max"], "median_rel_err": err["median"]}}


def scaled_errors(a, ref):
    """|a - ref| / max(|ref|, rms(ref)) per amplitude (the rms floor keeps tiny amplitudes of
    the Porter-Thomas tail from dominating): max and median."""
    import numpy as np

    a, ref = np.ravel(a), np.ravel(ref)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    e = np.abs(a - ref) / np.maximum(np.abs(ref), rms)
    return {"max": float(e.max()), "median": float(np.median(e))}


def run_sampling(amps7, amp_rate):
    """Fast frugal rejection sampling (one bit-string per 64-amplitude open batch, M = 10):
    the sampler's kernels on 2^20 synthetic Porter-Thomas batches of the 7x7 open batch (about
    the paper's 10^6 samples), then on the 7x7 workload's own amplitudes.  Its parity with the
    oracle is tested in tests/test_gpu_sampling.py."""
    import math

    import numpy as np
    import torch

    import rqc_inputs as R
    from paper_1811_09599_amd import frugal_sample

    n_q, m, nb, blen = 49, 10.0, 1 << 20, 64
    amps = torch.from_numpy(R.porter_thomas_amplitudes(nb, blen, n_q, 6100)).cuda()
    order_h, u_h = R.sampling_draws(nb, blen, blen, 6200)
    order, u = torch.from_numpy(order_h).cuda(), torch.from_numpy(u_h).cuda()
    acc, tail = frugal_sample(amps, order, u, n_q, m)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        frugal_sample(amps, order, u, n_q, m, sync=False)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    rate = float((acc >= 0).float().mean().item())
    # algorithmic bytes: every amplitude read once, one round of 64 visits (order + u) per
    # batch, the accepted value and the batch's partial sum written
    by = nb * (blen * 16 + 64 * 12 + 4 + 8)
    # paper's batch acceptance 1 - (1 - 1/M)^N_C; exact Porter-Thomas values for comparison
    paper_acc = 1 - (1 - 1 / m) ** blen
    pt_acc = 1 - (1 - (1 - math.exp(-m)) / m) ** blen
    o7, u7 = R.sampling_draws(amps7.shape[0], blen, blen, 6300)
    acc7, tail7 = frugal_sample(amps7, torch.from_numpy(o7).cuda(), torch.from_numpy(u7).cuda(),
                                n_q, m)
    del amps, order, u
    return {"workload": "frugal rejection sampling, M = 10, the 64 open-qubit values of each "
                        "batch visited in random order; 2^20 synthetic Porter-Thomas batches "
                        "(n = 49)",
            "metric": "samples/s", "value": rate * nb / sec, "unit": "samples/s",
            "batches_per_s": nb / sec, "ms_per_call": 1e3 * sec,
            "roofline": {"bound": "hbm", "achieved": round(by / sec / 1e9, 1),
                         "peak": PEAK["hbm"][0], "unit": "GB/s",
                         "frac": round(by / sec / 1e9 / PEAK["hbm"][0], 4), "traffic": None},
            "acceptance": rate, "acceptance_paper_formula": paper_acc,
            "acceptance_porter_thomas": pt_acc,
            "tail_error": tail, "tail_error_porter_thomas": (m + 1) * math.exp(-m),
            "on_7x7_amplitudes": {"batches": int(amps7.shape[0]),
                                  "accepted": int((acc7 >= 0).sum().item()),
                                  "tail_error": tail7,
                                  "samples_per_s_at_headline_rate": amp_rate / blen * paper_acc}}


def grid_cuts(circ):
    from paper_1811_09599_amd import plan_describe
    return plan_describe(circ)["cuts"]


def run_gradient(args):
    """Linear-XEB gradients of a batch of 96 fSim circuits (one contract_grad call = one step).
    Returns the result and, for the parity check of the CPU leg, the first 4x4 circuit with
    its bit-strings, fSim angle gradients and cross-entropy."""
    import numpy as np
    import torch

    import rqc_inputs as R
    from paper_1811_09599_amd import build_grid

    circs = R.fsim_batch(96, depth=12, sizes=(4, 5, 6), seed=5000, jitter_seed0=5900)
    bits = [R.bitstrings(c["n_qubits"], 128, 5500 + i) for i, c in enumerate(circs)]
    t0 = time.time()
    grid = build_grid(circs, autotune=not args.no_autotune)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    steps = max(1, min(args.steps, 2))
    for _ in range(max(args.warmup, 0)):
        grid.contract_grad(bits)
    torch.cuda.synchronize()
    grid.set_profiling(True)
    t0 = time.perf_counter()
    flops = 0.0
    for _ in range(steps):
        res = grid.contract_grad(bits)
        flops += grid.last_stats()["flops"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = grid.profile_read()
    grid.set_profiling(False)
    dom, roof = roofline(prof)
    top = sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:6]
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                   "gbps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in top}
    i4 = next(i for i, c in enumerate(circs) if c["n_qubits"] == 16)
    fsim = [j for j, gt in enumerate(circs[i4]["gates"]) if gt["kind"] == "fsim"]
    check = (i4, circs[i4], bits[i4], res["grad_params"][i4][fsim], float(res["loss"][i4]))
    sizes = np.bincount([c["n_qubits"] for c in circs])
    return {"workload": "96 fSim circuits, grids 4x4..6x6 (rows, cols from {4,5,6}), depth "
                        "1+12+1, theta = pi/2 + N(0, 0.02), phi = pi/6 + N(0, 0.02), linear "
                        "XEB over 128 bit-strings each; amplitudes and d/d(theta, phi) of every "
                        "fSim gate in one call per step",
            "metric": "circuits/s", "value": len(circs) * steps / dt, "unit": "circuits/s",
            "steps": steps, "ms_per_step": 1e3 * dt / steps,
            "qubits_histogram": {str(n): int(k) for n, k in enumerate(sizes) if k},
            "tflops": flops / dt / 1e12, "dominant_kernel": dom, "roofline": roof,
            "kernels": kernels, "grid_build_s": build_s}, check


def cpu_baseline(circ, grids, bits, open_q, n_slices, rows, cols):
    """The FP64 oracle (E2) on a bounded sample: n_slices slices of one bit-string batch,
    extrapolated to all slices; plus each precision's error against it on the same slices."""
    import numpy as np
    import torch

    from oracle import metrics
    from oracle import tn as E2

    grid = next(iter(grids.values()))
    S = grid.num_slices()
    ids = sorted(set(int(round(x)) for x in np.linspace(0, S - 1, n_slices)))
    cuts = grid.plan_cuts()
    net = E2.Network(circ)
    t0 = time.perf_counter()
    with torch.no_grad():
        ref = net.amplitudes(bits, open_q, cuts=cuts, slice_ids=ids,
                             order=E2.quadrant_order(rows, cols)).numpy()
    dt = time.perf_counter() - t0
    parity = {"slices": ids, "amplitudes": int(ref.size)}
    for p, g in grids.items():
        gpu = g.contract_amplitudes(bits, slice_ids=ids).cpu().numpy()
        err = metrics.amp_errors(gpu, ref, rows * cols)
        parity[p] = {"max_rel_err": err["max"], "median_rel_err": err["median"],
                     "l2_rel_err": err["l2"], "tol": TOL[p]}
    per_slice = dt / len(ids)
    rate = 64.0 / (per_slice * S)
    return {"cpu_baseline": {"value": rate, "unit": "amplitudes/s",
                             "cores": torch.get_num_threads(), "kind": "oracle",
                             "sample": "%d of %d slices of one 64-amplitude batch (FP64 tensor "
                                       "network, no reuse across slices), %.1f s; rate "
                                       "extrapolated to all %d slices" % (len(ids), S, dt, S)},
            "parity": parity}


def gradient_parity(i, circ, bits, grad, loss):
    """CPU leg: the gradient workload's circuit i against the FP64 state-vector adjoint."""
    from oracle import metrics
    from oracle import statevector as E1

    f_ref, g_ref = E1.linear_xeb_grad(circ, bits)
    return {"circuit": i, "oracle": "state-vector adjoint (FP64)",
            "grad_rel_l2": metrics.rel_l2(grad, g_ref), "loss_abs_err": abs(loss - f_ref),
            "tol": 1e-3}


if __name__ == "__main__":
    main()
