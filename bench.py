"""Throughput of the RQC amplitude contraction on one MI355X.

Headline workload: 7x7 grid, depth 1+40+1 (bond dimension 32 on every link), the quadrant
plan of SI A with 2 cut bonds (1024 slices; the largest intermediate 2^30 complex elements), a
6-qubit open batch (64 amplitudes per bit-string), fidelity f = 1/64 as 16 of the 1024 slices
(a block subset: one right-cut value and 16 bottom-cut values, SplitMix64-seeded), complex64
products on FP32 MFMA with FP64 slice sums.

A full 64-amplitude batch at f = 1/64 is ~5.8e15 flop (~40 s in complex64), so one step is one
slice of one bit-string's batch: a contraction call that adds that slice's 64 partial
amplitudes into the batch (accumulating output).  The library keeps the intermediates that do
not depend on the bottom cut across calls, so 16 consecutive steps cost what one call over the
16 slices costs.  Steps walk through the 16 slices of bit-string 0, then of bit-string 1, ...;
`value` is amplitudes/s at fidelity 1/64 = 64 / 16 = 4 amplitudes per step.

Split-bf16 and split-fp16 run the same steps and are reported alongside (`precisions`), each
with its error against complex64 on the accumulated batches.  The line also carries the
roofline of the dominant kernel (HIP events around every launch of the timed region, on the
launching stream; 8 real flops per complex multiply-add), the 4x4 1+16+1 workload (latency
bound: 256 amplitudes per call, eager and graph-replayed) and the CPU oracle timed on a bounded
sample.  Further workloads are opt-in (--extra).

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--extra gradient,diamond,...]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: dense MFMA fp32 / bf16 / fp16, fp32 vector without packed math, HBM3E
PEAK = {"mfma_fp32": (157.3, "TFLOP/s"), "mfma_bf16": (2500.0, "TFLOP/s"),
        "mfma_fp16": (2500.0, "TFLOP/s"),
        "alu": (78.6, "TFLOP/s"), "hbm": (8000.0, "GB/s")}
C64_TOL = 1e-5
# stated bounds of the 2^(n/2)-scaled amplitude error (max over the batch): split-bf16 at bond
# dimension 16 / 32, split-fp16 on random circuits
TOL = {"split_bf16": 2e-4, "split_bf16_d32": 1.5e-3, "split_fp16": 4 * C64_TOL, "c64": C64_TOL}
DTYPE = {"split_bf16": "bf16x3", "split_fp16": "fp16x3", "c64": "c64"}
EXTRAS = ("cfg2", "fsim", "sampling", "gradient", "diamond", "ceilings")

# headline workload (seeds: circuit 3000, bit-strings PCG64 3500, slices SplitMix64 3700)
ROWS = COLS = 7
DEPTH = 40
OPEN_PATCH = [(5, 0), (5, 1), (5, 2), (6, 0), (6, 1), (6, 2)]
FIDELITY = 1.0 / 64


# key of the headline workload in the committed HBM-traffic summaries
HEADLINE_WORKLOAD = "7x7_depth40_bond32_f1-64"


def flop_peak(name):
    """The arithmetic peak a kernel's algorithmic flops are measured against, from its name:
    a product is priced at the peak of the MFMA type it runs on."""
    if name.startswith(("gemm_split_bf16", "gemm_split3m_bf16")):
        return "mfma", PEAK["mfma_bf16"][0]
    if name.startswith(("gemm_split_fp16", "gemm_split3m_fp16")):
        return "mfma", PEAK["mfma_fp16"][0]
    if name.startswith(("gemm_mfma", "gemm_rows_mfma", "gemm_reduce_mfma")):
        return "mfma", PEAK["mfma_fp32"][0]
    if name.startswith("gemm_"):  # SIMT, rows, reduce and short-K products: FP32 vector ALU
        return "alu", PEAK["alu"][0]
    return None, None


def mfma_work_factor(name):
    """MFMA flops the kernel issues per algorithmic flop (8 per complex multiply-add): the
    split product of complex parts hi+lo runs 3 real products (hi.hi, hi.lo, lo.hi) per real
    product of the 4-multiplication form; the 3-multiplication (Gauss) form runs 3 real
    products per complex one instead of 4."""
    if name.startswith("gemm_split3m"):
        return 2.25
    if name.startswith("gemm_split"):
        return 3.0
    if name.startswith("gemm_mfma3m"):
        return 0.75
    return 1.0


def roofline(prof, workload=None):
    """Roofline of the kernel with the most time: its algorithmic flops (8 per complex
    multiply-add) and bytes per launch, recorded by the library with each launch, over its
    average launch time; the bound is the resource the kernel uses the larger fraction of.
    `traffic` is the counted HBM bytes per launch of that kernel on `workload`, if measured."""
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
    r = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
         "frac": round(achieved / peak, 4), "traffic": measured_traffic(name, workload),
         "flop_frac": round(flop_frac, 4), "hbm_frac": round(hbm_frac, 4),
         "avg_launch_us": round(1e3 * k["ms"] / max(k["launches"], 1), 3),
         "launches": k["launches"],
         "flops_per_launch": k["flops"] / max(k["launches"], 1)}
    f = mfma_work_factor(name)
    if f != 1.0:
        r["mfma_instruction_tflops"] = round(tflops * f, 1)
        r["mfma_instruction_frac"] = round(tflops * f / fpeak, 4)
    return name, r


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summaries
    (profiles/hbm_traffic_*.md, lines "traffic <workload> <kernel> <bytes per launch>
    <source> <sha256 of source>", from two rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE,
    scaled by what the counters read for a 1 GiB device copy), or None when there is none for
    that pair or the kernel's source has changed since."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        with open(path) as f:
            for line in f:
                w = line.split()
                if (len(w) == 6 and w[0] == "traffic" and w[1] == workload
                        and w[2] == kernel):
                    src = os.path.join(ROOT, w[4])
                    if not os.path.exists(src):
                        return None
                    with open(src, "rb") as fs:
                        if hashlib.sha256(fs.read()).hexdigest() != w[5]:
                            return None
                    return float(w[3])
    return None


def kernel_table(prof, top=8):
    return {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                "avg_us": round(1e3 * v["ms"] / max(v["launches"], 1), 3),
                "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                "gbps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)}
            for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:top]}


def scaled_errors(a, ref):
    """|a - ref| / max(|ref|, rms(ref)) per amplitude (the rms floor keeps tiny amplitudes of
    the Porter-Thomas tail from dominating): max and median."""
    import numpy as np

    a, ref = np.ravel(a), np.ravel(ref)
    if a.size != ref.size:
        raise ValueError("size mismatch")
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    e = np.abs(a - ref) / np.maximum(np.abs(ref), rms)
    return {"max": float(e.max()), "median": float(np.median(e))}


def headline_inputs():
    import rqc_inputs as R
    circ = R.grid_rqc(ROWS, COLS, DEPTH, 3000)
    open_q = R.grid_ids((ROWS, COLS), OPEN_PATCH)
    bits = R.bitstrings(ROWS * COLS, 256, 3500, open_q)
    return circ, open_q, bits


def run_headline(precision, circ, open_q, bits, ids, args):
    """W + K steps of the headline workload in one precision; returns the accumulated batches
    (torch complex128 [bit-strings touched, 64]) and the timing of the K timed steps."""
    import torch

    from paper_1811_09599_amd import build_grid

    t0 = time.time()
    grid = build_grid(circ, open_qubits=open_q, precision=precision, slice_mode="block",
                      bitstring_batch=1, autotune=args.autotune)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    k = len(ids)
    n_steps = args.warmup + args.steps
    outs = torch.zeros(((n_steps + k - 1) // k, 64), dtype=torch.complex128, device="cuda")

    def step(i):
        j, s = divmod(i, k)
        grid.contract_amplitudes(bits[j:j + 1], slice_ids=[ids[s]], out=outs[j:j + 1],
                                 accumulate=True)
        return grid.last_stats()["flops"]

    t0 = time.time()
    warm_flops = 0.0
    for i in range(args.warmup):
        warm_flops += step(i)
    torch.cuda.synchronize()
    warm_s = time.time() - t0
    grid.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flops = 0.0
    for i in range(args.warmup, n_steps):
        flops += step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = grid.profile_read()
    grid.set_profiling(False)
    grid.close()
    dom, roof = roofline(prof, HEADLINE_WORKLOAD)
    amps = args.steps * 64.0 / k  # fidelity-f amplitudes completed
    print("[bench] %s: %d steps in %.2f s (warm-up %.1f s, grid build %.1f s)"
          % (precision, args.steps, dt, warm_s, build_s), file=sys.stderr, flush=True)
    return outs, {"value": amps / dt, "ms_per_step": 1e3 * dt / args.steps,
                  "tflops": flops / dt / 1e12, "timed_flops": flops,
                  "dominant_kernel": dom, "roofline": roof, "kernels": kernel_table(prof),
                  "grid_build_s": round(build_s, 3), "warmup_s": round(warm_s, 3)}


def run_cfg1(args):
    """4x4, depth 1+16+1, 256 seeded bit-strings per call (all of them in one call), complex64,
    no cuts: the latency-bound configuration, eager and replayed from a HIP graph."""
    import torch

    import rqc_inputs as R
    from paper_1811_09599_amd import build_grid

    circ = R.grid_rqc(4, 4, 16, 1001)
    # two sets of 256 bit-strings, alternated: a call never repeats the previous call's
    # bit-strings, so every call contracts (nothing is kept from the call before)
    sets = [R.bitstrings(16, 256, 1500), R.bitstrings(16, 256, 1501)]
    res = {"workload": "4x4 RQC depth 1+16+1, 256 amplitudes per call (no cuts), complex64",
           "metric": "amplitudes/s", "unit": "amplitudes/s"}
    reps = max(50, 10 * args.steps)
    # both modes on a stream of their own: a graph is captured and replayed on the caller's
    # stream (the null stream would put a second stream and two events around every call)
    side = torch.cuda.Stream()
    for mode in ("eager", "graph"):
        with torch.cuda.stream(side):
            g = build_grid(circ, graph=(mode == "graph"))
            out = torch.empty((256, 1), dtype=torch.complex128, device="cuda")
            for i in range(3):
                g.contract_amplitudes(sets[i % 2], out=out)
            side.synchronize()
            flops = 0.0
            t0 = time.perf_counter()
            for i in range(reps):
                g.contract_amplitudes(sets[i % 2], out=out)
                flops += g.last_stats()["flops"]
            side.synchronize()
            dt = time.perf_counter() - t0
        res[mode] = {"value": 256.0 * reps / dt, "ms_per_call": 1e3 * dt / reps,
                     "calls": reps, "flops_per_call": flops / reps}
        g.close()
    res["value"] = max(res["eager"]["value"], res["graph"]["value"])
    return res


def cpu_info():
    """Host CPU model, physical cores (distinct (package, core) pairs) and logical CPUs."""
    model, pairs, logical, phys, core = "unknown", set(), 0, None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                    pairs.add((phys, core))
    except OSError:
        pass
    return {"cpu_model": model, "physical_cores": len(pairs) or None, "logical_cpus": logical,
            "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(circ_h, open_q, step_flops_fresh, k, budget_s):
    """The FP64 oracle (E2, torch complex128 on the host cores) on a bounded sample: single
    slices of one 64-amplitude batch of the 7x7 depth 1+32+1 circuit (bond dimension 16; the
    oracle cannot hold a bond-32 slice's 2^30-element tensors in complex128 within the time
    budget), as many as fit the budget.  Its rate under the plan's flop count (a slice
    contracted from scratch, as the oracle does) is applied to the headline's slice, giving the
    oracle's amplitudes/s at f = 1/64 (an extrapolation, stated as such).  The same slices are
    contracted on the GPU in complex64 and compared with the oracle (parity at full 7x7 size)."""
    import numpy as np
    import torch

    import rqc_inputs as R
    from oracle import metrics
    from oracle import tn as E2
    from paper_1811_09599_amd import build_grid, plan_describe

    circ = R.grid_rqc(ROWS, COLS, 32, 2000)
    bits = R.bitstrings(ROWS * COLS, 1, 2500, open_q)
    plan = plan_describe(circ, open_qubits=open_q)
    slice_flops = float(sum(s["flops"] for s in plan["steps"]))
    grid = build_grid(circ, open_qubits=open_q)
    cuts = grid.plan_cuts()
    S = grid.num_slices()
    net = E2.Network(circ)
    order = E2.quadrant_order(ROWS, COLS)
    cand = [37, 200, 113, 250, 5, 166, 81, 222]
    done, times, par = [], [], []
    t_all = time.perf_counter()
    with torch.no_grad():
        for sid in cand:
            t0 = time.perf_counter()
            ref = net.amplitudes(bits, open_q, cuts=cuts, slice_ids=[sid], order=order).numpy()
            times.append(time.perf_counter() - t0)
            done.append(sid)
            gpu = grid.contract_amplitudes(bits, slice_ids=[sid]).cpu().numpy()
            par.append(metrics.amp_errors(gpu, ref, ROWS * COLS))
            if time.perf_counter() - t_all > budget_s and len(done) >= 2:
                break
    grid.close()
    t_slice = float(np.mean(times))
    gflops = slice_flops / t_slice / 1e9
    # the oracle contracts every slice from scratch: one fidelity-f batch = k such slices
    t_batch = k * step_flops_fresh / (gflops * 1e9)
    info = cpu_info()
    return {"value": 64.0 / t_batch, "unit": "amplitudes/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": "%d single slices (ids %s of %d) of one 64-amplitude batch of the 7x7 "
                      "depth 1+32+1 circuit (bond dim 16), FP64 tensor network, %.1f s in all, "
                      "%.2f s per slice = %.1f GFLOP/s under the plan's count (%.3g flop per "
                      "slice from scratch); extrapolated to the headline's slice (%.3g flop from "
                      "scratch) x %d slices per fidelity-1/64 batch" %
                      (len(done), done, S, float(np.sum(times)), t_slice, gflops, slice_flops,
                       step_flops_fresh, k),
            "oracle_gflops": round(gflops, 2), **info,
            "parity_c64_vs_oracle_d16": {
                "slices": done, "max_rel_err": max(p["max"] for p in par),
                "median_rel_err": float(np.median([p["median"] for p in par])),
                "l2_rel_err": max(p["l2"] for p in par), "tol": C64_TOL}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="all",
                    choices=["all", "c64", "split_bf16", "split_fp16"])
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work in the CPU baseline (at least 2 slices)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cfg1", action="store_true", help="skip the 4x4 workload")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time kernel variants per step on first use (default: "
                         "its shape rules)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="shape rules in the opt-in workloads too")
    ap.add_argument("--extra", default="",
                    help="comma-separated opt-in workloads: " + ",".join(EXTRAS) + " or all")
    ap.add_argument("--bitstrings", type=int, default=8,
                    help="bit-strings per step of the opt-in cfg2/fsim workloads")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device to device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested; see the sharding design)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    extras = set(EXTRAS) if args.extra == "all" else {e for e in args.extra.split(",") if e}
    if extras - set(EXTRAS):
        print("unknown --extra workloads: %s" % sorted(extras - set(EXTRAS)), file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1811_09599_amd import plan_describe, select_slices

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
    ceil = ceilings() if "ceilings" in extras else None
    circ, open_q, bits = headline_inputs()
    plan = plan_describe(circ, open_qubits=open_q)
    S = plan["num_slices"]
    ids = select_slices(S, FIDELITY, 3700, "block")
    k = len(ids)
    step_fresh = float(sum(s["flops"] for s in plan["steps"]))
    precs = ["c64", "split_bf16", "split_fp16"] if args.precision == "all" else [args.precision]
    results, outs = {}, {}
    for p in precs:
        outs[p], results[p] = run_headline(p, circ, open_q, bits, ids, args)
        outs[p] = outs[p].cpu().numpy()
    head = precs[0]
    r = results[head]
    res = {
        "metric": "amplitudes/s", "value": r["value"], "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[head], "data": "synthetic",
        "config": {"workload": "7x7 RQC depth 1+40+1 (bond dim 32), quadrant plan with 2 cuts "
                               "(%d slices, largest intermediate 2^%d), fidelity 1/64 = %d "
                               "slices (block subset %d..%d), 6-qubit open batch (64 "
                               "amplitudes per bit-string); one step = one slice of one "
                               "bit-string's batch (accumulating call, intermediates kept "
                               "across calls), value = amplitudes/s at fidelity 1/64"
                               % (S, plan["max_bits"], k, ids[0], ids[-1]),
                   "grid": "7x7", "depth": "1+40+1", "bond_dim": 32, "slices": S,
                   "fidelity": FIDELITY, "slice_ids": [int(i) for i in ids],
                   "amplitudes_per_bitstring": 64, "bitstrings_touched": int(outs[head].shape[0]),
                   "flops_per_slice_from_scratch": step_fresh, "precision": head},
        "tflops": r["tflops"], "dominant_kernel": r["dominant_kernel"],
        "roofline": r["roofline"], "kernels": r["kernels"],
        "precisions": {p: {kk: v for kk, v in results[p].items() if kk != "kernels"}
                       for p in precs},
    }
    if head == "c64":
        res["tflops_frac_fp32_mfma_peak"] = r["tflops"] / PEAK["mfma_fp32"][0]
    # the paper's CPU clusters, as context only (Results; table of effective runtimes of one
    # perfect-fidelity amplitude): a different machine and a different unit of work
    res["paper_context"] = {
        "clusters_peak_tflops_fp32": 20000.0,
        "clusters_peak_note": "NASA Pleiades + Electra combined, single precision, 64% of their "
                              "achievable peak",
        "this_gpu_tflops_over_clusters_peak": r["tflops"] / 20000.0,
        "perfect_fidelity_amplitude_7x7_d40_s": {"pleiades": 1.22e-2 * 3600,
                                                 "electra": 1.16e-2 * 3600},
        "this_gpu_all_1024_slices_s_estimate": {
            p: 1024.0 * results[p]["ms_per_step"] / 1e3 for p in precs},
        "note": "estimate = 1024 slices x this run's ms per step (a slice of one 64-amplitude "
                "batch, slice-independent intermediates kept); not measured end to end",
    }
    for p in precs:
        if p != "c64" and "c64" in results:
            res["precisions"][p]["speedup_vs_c64"] = results[p]["value"] / results["c64"]["value"]
            e = scaled_errors(outs[p], outs["c64"])
            tol = TOL["split_bf16_d32"] if p == "split_bf16" else TOL[p]
            res["precisions"][p]["vs_c64"] = {"max_rel_err": e["max"],
                                              "median_rel_err": e["median"], "tol": tol,
                                              "amplitudes": int(outs[p].size)}
    if not args.no_cfg1:
        res["cfg1_4x4"] = run_cfg1(args)
    # the opt-in workloads take a few steps each, whatever the headline's count
    xargs = argparse.Namespace(**vars(args))
    xargs.steps, xargs.warmup = min(args.steps, 3), min(args.warmup, 1)
    args = xargs
    if "cfg2" in extras:  # the plain complex64 path of that configuration, and split-bf16
        res["cfg2_7x7_d16"] = run_cfg2(args, "c64")
        res["cfg2_7x7_d16_split_bf16"] = run_cfg2(args, "split_bf16")
    if "fsim" in extras:
        res["fsim_7x7"] = run_fsim(args, "split_bf16")
    if "sampling" in extras:
        res["sampling"] = run_sampling_leg(args)
    grad_check = None
    if "gradient" in extras:
        res["gradient"], grad_check = run_gradient(args)
    if "diamond" in extras:
        res["diamond"] = run_diamond(args)
    if ceil:
        res["ceilings"] = ceil
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(circ, open_q, step_fresh, k, args.cpu_budget)
        if grad_check is not None:
            res["gradient"]["parity"] = gradient_parity(*grad_check)
    print(json.dumps(res), flush=True)


def run_cfg2(args, precision):
    """7x7 depth 1+32+1 (bond dim 16), all 256 slices, --bitstrings per step."""
    import rqc_inputs as R
    circ = R.grid_rqc(ROWS, COLS, 32, 2000)
    open_q = R.grid_ids((ROWS, COLS), OPEN_PATCH)
    all_bits = R.bitstrings(ROWS * COLS, 1024, 2500, open_q)
    g, r = run_precision(precision, circ, open_q, all_bits, args)
    g.close()
    return {"workload": "7x7 RQC depth 1+32+1 (bond dim 16), all 256 slices, %d bit-strings "
                        "per step, %s" % (args.bitstrings, precision),
            "metric": "amplitudes/s", "unit": "amplitudes/s",
            **{kk: r[kk] for kk in ("value", "ms_per_step", "tflops", "dominant_kernel",
                                    "roofline")}}


def run_fsim(args, precision):
    """fSim couplers at half the depth: the same bond dimensions, plan and flops (1+t/2+1)."""
    import rqc_inputs as R
    circ_f = R.grid_rqc(ROWS, COLS, 16, 2002, two_qubit="fsim", jitter_sd=0.02, jitter_seed=3)
    open_q = R.grid_ids((ROWS, COLS), OPEN_PATCH)
    all_bits = R.bitstrings(ROWS * COLS, 1024, 2500, open_q)
    g, r = run_precision(precision, circ_f, open_q, all_bits, args)
    g.close()
    return {"workload": "7x7 RQC with fSim(pi/2 + N(0, 0.02), pi/6 + N(0, 0.02)) couplers, "
                        "depth 1+16+1 (bond dim 16), all 256 slices, %s" % precision,
            "metric": "amplitudes/s", "unit": "amplitudes/s",
            **{kk: r[kk] for kk in ("value", "ms_per_step", "tflops", "dominant_kernel",
                                    "roofline")}}


def run_sampling_leg(args):
    import rqc_inputs as R
    from paper_1811_09599_amd import build_grid
    circ = R.grid_rqc(ROWS, COLS, 32, 2000)
    open_q = R.grid_ids((ROWS, COLS), OPEN_PATCH)
    bits = R.bitstrings(ROWS * COLS, 4, 2500, open_q)
    g = build_grid(circ, open_qubits=open_q, precision="split_bf16")
    a = g.contract_amplitudes(bits)
    g.close()
    return run_sampling(a, None)


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

    flops = 8.0 * m ** 3 * b  # algorithmic: 8 per complex multiply-add
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
        chunk = all_bits[lo:lo + B]
        grid.contract_amplitudes(chunk, out=out[:len(chunk)])
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
                                  "samples_per_s_at_headline_rate":
                                      None if amp_rate is None else amp_rate / blen * paper_acc}}


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
    t0 = time.perf_counter()
    flops = 0.0
    for _ in range(steps):
        res = grid.contract_grad(bits)
        flops += grid.last_stats()["flops"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # one more call with every launch timed by events (they add their own overhead)
    grid.set_profiling(True)
    grid.contract_grad(bits)
    prof = grid.profile_read()
    grid.set_profiling(False)
    dom, roof = roofline(prof)
    top = sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:6]
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                   "gbps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)} for k, v in top}
    grid.close()
    # the same calls replayed from a HIP graph (one slice per circuit: captured by the second
    # call, after the first has tuned), on a stream of their own, and checked against eager
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        gg = build_grid(circs, autotune=not args.no_autotune, graph=True)
        for _ in range(2):
            gg.contract_grad(bits)
        side.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rg = gg.contract_grad(bits)
        side.synchronize()
        dt_graph = time.perf_counter() - t0
        gg.close()
    graph_err = max(float(np.linalg.norm(rg["grad_params"][i] - res["grad_params"][i]) /
                          max(np.linalg.norm(res["grad_params"][i]), 1e-300))
                    for i in range(len(circs)))
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
            "kernels": kernels, "grid_build_s": build_s,
            "graph": {"value": len(circs) * steps / dt_graph, "ms_per_step": 1e3 * dt_graph / steps,
                      "max_grad_rel_diff_vs_eager": graph_err}}, check


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
