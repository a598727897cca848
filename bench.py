"""Benchmark of the string-method hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

One step = one string iteration over every image of the workload: field of
every image (FFT dipolar convolution + exchange/DMI/anisotropy stencils),
FP64 energies, projected descent step with renormalisation, FP64 arc
lengths, reparametrisation.  The headline value is site-field evaluations
per second of the FP32-mixed form replayed as a HIP graph; the FP64 plain
form (direct launches) runs the same workload for the speed-up and the
barrier difference.  Inputs are synthetic (seeded skyrmion-tube string) and
already resident in HBM when timing starts.  Prints one JSON line.
"""
import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "site-field evals/s + string iters/s; FP32-batched vs FP64 plain at 1e-4 barrier"
HBM_PEAK_GBS = 8000.0
# FP32 vector ceiling of the instructions these kernels issue: 256 CUs x 4 SIMDs
# x 16 lanes x 2 flops per FMA x 2.4 GHz (the published 157.3 TFLOP/s counts
# packed FP32, which these kernels are compiled without)
FP32_VECTOR_NONPACKED_TFLOPS = 78.6
KERNEL_SOURCES = ["paper_1804_07135_amd/csrc/ssm_kernels.hip", "paper_1804_07135_amd/csrc/ssm_internal.hpp",
                  "paper_1804_07135_amd/csrc/ssm_fft.hpp", "paper_1804_07135_amd/csrc/ssm_api.hip"]
_CODE_TOKENS = re.compile(r'//[^\n]*|/\*.*?\*/|("(?:\\.|[^"\\])*")', re.S)


def kernel_source_hash():
    """Hash of the code of the kernels and of their launch configuration
    (comments and layout ignored): a profile is reused only while this is
    unchanged."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            code = _CODE_TOKENS.sub(lambda m: m.group(1) or " ", fh.read())
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def half_len(n, axis="x", nz=1):
    """The documented half padded length of the x or y axis (the same rule
    for both, any layer count): the power of two >= n, or for n > 32 the
    length 3 2^a >= n (a >= 4, at most 768) when that is smaller."""
    p2 = 1 << (n - 1).bit_length()
    t = 48
    while t < n:
        t *= 2
    return t if n > 32 and t < p2 and t <= 768 else p2


def algorithmic_bytes(w, ts):
    """Bytes each kernel must move per launch (one iteration), spin scalar size ts."""
    nx, ny, nz, K = w["nx"], w["ny"], w["nz"], w["K"]
    mx, my = half_len(nx, "x"), half_len(ny, "y", nz)
    pz = 1 if nz == 1 else 2 * (1 << (nz - 1).bit_length())
    N = nx * ny * nz
    spins = K * 3 * N * ts                         # one string
    xspec = K * (mx + 1) * 3 * nz * ny * 2 * ts    # x half-spectra of one string
    nhat = (mx + 1) * 2 * my * pz * 6 * ts         # dipole-kernel spectrum
    return {
        "k_xfwd": spins + xspec,
        "k_conv": 2 * xspec + nhat,
        "k_xinv": xspec + 2 * spins,
        "k_arc": spins,
        # every source image read once (consecutive targets share their
        # sources), every image of the new string written once
        "k_interp": 2 * spins,
    }


def replay_chunk(warmup, graph_chunk):
    """Iterations per replayed HIP graph for a run with `warmup` untimed
    steps: graph capture and instantiation happen in the warm-up, never in
    the timed steps, so the chunk is at most the warm-up's length (no
    warm-up: 0, direct launches)."""
    return graph_chunk if warmup >= graph_chunk else max(warmup, 0)


def time_iterations(sm, steps, tau):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sm.iterate(steps, tau)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp():
    """The OpenMP runtime the oracle library runs on (same process)."""
    import ctypes
    for name in ("libgomp.so.1", "libgomp.so"):
        try:
            lib = ctypes.CDLL(name)
            lib.omp_get_max_threads.restype = ctypes.c_int
            return lib
        except OSError:
            continue
    return None


def _sample_rate(oracle, w, s0, budget_s, seed):
    """Direct-sum fields at random sites of image 0 for about budget_s."""
    import numpy as np
    N = w["nx"] * w["ny"] * w["nz"]
    rng = np.random.default_rng(seed)
    n, t = 16, 0.0
    while True:
        sites = rng.choice(N, size=n, replace=False)
        t0 = time.perf_counter()
        oracle.field_at(s0[0], w["J"], w["d"], w["ku"], w["D"], sites)
        t = time.perf_counter() - t0
        if t > budget_s / 2 or n >= N:
            return n, t
        n = min(N, int(n * max(2.0, 0.75 * budget_s / max(t, 1e-3))))


def cpu_baseline(w, s0, budget_s):
    """The oracle (direct O(N^2) dipole sum, FP64, OpenMP), as it stands,
    timed on this host: fields at a sample of sites of image 0 of the
    workload with every host thread and with one thread, and the full
    200-iteration run of the 32x32x1, 10-image workload with every thread."""
    from oracle import oracle
    from paper_1804_07135_amd import inputs
    oracle.build()
    omp = _omp()
    threads = omp.omp_get_max_threads() if omp else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n, t = _sample_rate(oracle, w, s0, budget_s, 0)
    out = {"value": n / t, "unit": "site-field evals/s", "cores": threads, "kind": "oracle",
           "sample": f"direct-sum fields at {n} random sites of image 0 of the "
                     f"{w['nx']}x{w['ny']}x{w['nz']} lattice ({t:.1f} s, {threads} threads)",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    if omp:
        omp.omp_set_num_threads(1)
        n1, t1 = _sample_rate(oracle, w, s0, budget_s / 3, 1)
        omp.omp_set_num_threads(threads)
        out["value_1_thread"] = n1 / t1
        out["sample_1_thread"] = f"{n1} sites ({t1:.1f} s)"
    c1 = dict(inputs.WORKLOADS["bloch_32x32x1_k10"])
    s1 = inputs.build_string(c1)
    t0 = time.perf_counter()
    oracle.iterate(s1, c1["J"], c1["d"], c1["ku"], c1["D"], c1["iters"], c1["tau"])
    t = time.perf_counter() - t0
    kn = c1["K"] * c1["nx"] * c1["ny"] * c1["nz"]
    # iterations plus the closing evaluation, one field per image each
    out["bloch_32x32x1_k10_full_run"] = {"iters": c1["iters"], "seconds": t, "threads": threads,
                                         "string_iters_per_s": c1["iters"] / t,
                                         "site_field_evals_per_s": (c1["iters"] + 1) * kn / t}
    return out


def _csv_rows(path):
    import csv
    import glob
    files = glob.glob(os.path.join(path, "**", "*.csv"), recursive=True)
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _kernel_key(name):
    for k in ("k_xfwd", "k_conv", "k_xinv", "k_arc", "k_reduce", "k_interp", "k_spec1", "k_spec2",
              "k_spec3", "copyBuffer"):
        if k in name:
            return k
    return None


def rk_leg(ssm, torch, prob, s0, KN, args):
    """The string iteration with the paper's integrator (adaptive Dormand-Prince
    5(4) over an interval per image), FP32-mixed form: one warm-up iteration,
    then args.rk_iters timed ones.  Every stage is a field evaluation of all
    images, so site-field evals/s counts K N per evaluation."""
    sm = ssm.StringMethod(prob, ssm.SSM_FP32_MIXED, with_rk=True)
    sm.set_integrator(ssm.SSM_STEP_DOPRI54, args.rk_tol, args.rk_tol, 0.1)
    sm.set_string(s0)
    sm.iterate(1, args.rk_interval)
    _, _, n0 = sm.rk_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sm.iterate(args.rk_iters, args.rk_interval)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    counts, _, n1 = sm.rk_stats()
    c = counts.cpu().numpy()
    res = {"interval": args.rk_interval, "rtol": args.rk_tol, "atol": args.rk_tol, "iters": args.rk_iters,
           "ms_per_iter": dt / args.rk_iters * 1e3, "string_iters_per_s": args.rk_iters / dt,
           "field_evals_per_iter": (n1 - n0) / args.rk_iters,
           "site_field_evals_per_s": (n1 - n0) * KN / dt,
           "accepted_steps_total": int(c[:, 0].sum()), "rejected_steps_total": int(c[:, 1].sum()),
           "barrier": float(sm.barrier().cpu().numpy()[0][0]), "flags": int(sm.check())}
    del sm
    torch.cuda.empty_cache()
    return res


def full_run_leg(ssm, torch, prob, s0, iters, tau, chunk):
    """The workload's full run in both forms from the same initial string
    (FP32-mixed replayed as graphs, FP64 plain with direct launches): the
    barrier of each after `iters` iterations and their relative difference
    (target 1e-4), with each form's time."""
    res = {"iters": iters}
    bars = {}
    for name, prec, gc in (("fp32_mixed", ssm.SSM_FP32_MIXED, chunk), ("fp64_plain", ssm.SSM_FP64, 0)):
        sm = ssm.StringMethod(prob, prec)
        sm.set_options(check_every=10, graph_chunk=gc)
        sm.set_string(s0)
        dt = time_iterations(sm, iters, tau)
        b = sm.barrier().cpu().numpy()[0]
        bars[name] = float(b[0])
        res[name] = {"barrier": float(b[0]), "argmax": int(b[1]), "ms_per_step": dt / iters * 1e3,
                     "flags": int(sm.check())}
        del sm
        torch.cuda.empty_cache()
    res["barrier_rel_err_fp32_vs_fp64"] = abs(bars["fp32_mixed"] - bars["fp64_plain"]) / abs(bars["fp64_plain"])
    return res


def small_workloads_leg(ssm, torch, inputs, steps, chunk):
    """Rates of the 32x32x1 (10 images) and 64x64x1 (20 images) workloads in
    both forms: FP64 plain (direct launches) and FP32-mixed (graph replay).
    Too small to fill the GPU; they run in L2 and are launch- and
    latency-bound."""
    res = {}
    for name in ("bloch_32x32x1_k10", "boundary_64x64x1_k20"):
        w = dict(inputs.WORKLOADS[name])
        prob = dict(nx=w["nx"], ny=w["ny"], nz=w["nz"], K=w["K"], J=w["J"], d=w["d"], ku=w["ku"], D=w["D"])
        s0 = inputs.build_string(w)
        kn = w["K"] * w["nx"] * w["ny"] * w["nz"]
        r = {}
        for form, prec, gc in (("fp64_plain", ssm.SSM_FP64, 0), ("fp32_mixed", ssm.SSM_FP32_MIXED, chunk)):
            sm = ssm.StringMethod(prob, prec)
            sm.set_options(check_every=10, graph_chunk=gc)
            sm.set_string(s0)
            sm.iterate(chunk, w["tau"])
            dt = time_iterations(sm, steps, w["tau"])
            r[form] = {"ms_per_step": dt / steps * 1e3, "string_iters_per_s": steps / dt,
                       "site_field_evals_per_s": steps * kn / dt}
            del sm
        r["speedup_fp32_vs_fp64"] = r["fp64_plain"]["ms_per_step"] / r["fp32_mixed"]["ms_per_step"]
        res[name] = r
    torch.cuda.empty_cache()
    return res


def sweep_leg(ssm, torch, inputs, args):
    """The (k_u, d) sweep: 64 points on lattices 48..96 (16 images each) in
    one FP32-mixed context, tiles from the autotuner, iterations replayed as
    HIP graphs, spline interpolation with the climbing image, run to a
    perpendicular-force norm of args.sweep_tol (cap args.sweep_iters).
    Reports which points converged, their barriers and envelope derivatives
    (NaN where not converged), the rate over the iterations each point ran,
    and the graph replay's time against the summed kernel time."""
    import tempfile
    import numpy as np
    from paper_1804_07135_amd import sweep
    pts = inputs.sweep_points()
    chunk = 100
    sm = ssm.StringMethod(sweep.sweep_problems(pts), ssm.SSM_FP32_MIXED)
    sm.set_options(check_every=chunk, graph_chunk=chunk)
    sm.set_reparam(ssm.SSM_INTERP_SPLINE, True)
    s0 = sweep.initial_strings(pts)
    sm.set_string(s0)
    with tempfile.TemporaryDirectory() as td:
        sm.autotune(os.path.join(td, "tiles.txt"))
    sm.set_string(s0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = sm.iterate(args.sweep_iters, 0.1, args.sweep_tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = it.cpu().numpy()
    bar = sm.barrier().cpu().numpy()
    _, fn = sm.tangents()
    force = fn.cpu().numpy()
    flags = sm.check()
    conv = sweep.converged_mask(force, args.sweep_tol) & np.isfinite(bar[:, 0])
    dB = sweep.mask_unconverged(bar[:, 2:6], conv)
    kn = np.array([p["K"] * p["nx"] * p["ny"] * p["nz"] for p in pts], dtype=np.float64)
    evals = float((iters * kn).sum())
    # graph replay against the kernels' own time on this many-small-problem
    # batch: the same 200 iterations replayed, then launched one by one with
    # HIP events around every kernel
    n = 200
    sm.set_string(s0)
    g = time_iterations(sm, n, 0.1) / n
    sm.profile(True)
    sm.profile_read()
    sm.set_string(s0)
    sm.iterate(n, 0.1)
    kern = sum(v[0] for v in sm.profile_read().values()) / n * 1e-3
    sm.profile(False)
    res = {"points": len(pts), "images_per_point": 16, "tol_force": args.sweep_tol, "max_iter": args.sweep_iters,
           "reparam": "spline + climbing image", "converged": int(conv.sum()), "seconds": dt,
           "iterations_max": int(iters.max()), "iterations_mean": float(iters.mean()),
           "site_field_evals_per_s": evals / dt, "flags": int(flags),
           "graph_ms_per_iter": g * 1e3, "kernel_ms_per_iter": kern * 1e3, "graph_gap_frac": (g - kern) / g,
           "per_point": [[int(p["nx"]), round(p["ku"], 4), round(p["d"], 4), bool(c), int(i), float(f),
                          float(b), float(dd[2]), float(dd[1])]
                         for p, c, i, f, b, dd in zip(pts, conv, iters, force, bar[:, 0], dB)],
           "per_point_columns": ["L", "ku", "d", "converged", "iters", "force", "barrier", "dB_dku", "dB_dd"]}
    del sm
    torch.cuda.empty_cache()
    return res


def paper_shape_leg(ssm, torch, args):
    """The paper's production shape: a 112x112x1 monolayer, 60 images, with
    its material in SI units (d = 5.30 meV, k = 0.5 meV), FP32-mixed form,
    graph replay, tiles from the autotuner: one problem alone, then
    args.paper_batch (d, k) points in one context (the batched
    phase-diagram form).  Explicit steps of 0.1
    (the paper's interval of 5e-14 s is 1.74 in these units at damping 1,
    for the adaptive integrator, whose cost the integrator leg gives)."""
    import tempfile
    from paper_1804_07135_amd import si
    res = {}
    tau = 0.1
    for n_points in (1, args.paper_batch):
        ds = [5.30 + 0.1 * i for i in range(n_points)]
        probs = [si.paper_problem(d, 0.5) for d in ds]
        strings = [si.initial_string("bloch", 112, 60, 10.0, seed=i) for i in range(n_points)]
        sm = ssm.StringMethod(probs, ssm.SSM_FP32_MIXED)
        sm.set_options(check_every=10, graph_chunk=10)
        sm.set_string(strings)
        with tempfile.TemporaryDirectory() as td:
            sm.autotune(os.path.join(td, "tiles.txt"))
        sm.set_string(strings)
        sm.iterate(10, tau)
        steps = args.paper_steps
        dt = time_iterations(sm, steps, tau)
        kn = n_points * 60 * 112 * 112
        res[f"points_{n_points}"] = {"ms_per_step": dt / steps * 1e3, "string_iters_per_s": steps / dt,
                                     "site_field_evals_per_s": steps * kn / dt, "flags": int(sm.check())}
        del sm
        torch.cuda.empty_cache()
    res.update({"lattice": [112, 112, 1], "images": 60, "tau": tau, "steps": args.paper_steps})
    return res


RDREQ = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")


def summarize_profiles(args):
    """Turn rocprofv3 outputs of the bench (and of the copy probe) into the
    committed summaries: per-kernel durations, and HBM traffic per kernel.

    Read bytes come from the L2-to-memory read requests by size (32, 64 and
    128 bytes: TCC_EA0_RDREQ_{32B,64B,128B}), write bytes from WRITE_SIZE
    (the write requests are 32 or 64 bytes).  The copy probe's passes, when
    present, check both against a copy of known size; FETCH_SIZE, whose
    formula takes 128-byte requests from TCC_BUBBLE, is reported beside the
    request-size count for comparison."""
    import statistics
    d = args.summarize_profiles
    w = args.workload
    stats = {}
    for r in _csv_rows(os.path.join(d, "trace")):
        if "Kernel_Name" in r and "Start_Timestamp" in r:
            k = _kernel_key(r["Kernel_Name"])
            if k:
                stats.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)

    def per_dispatch(sub):
        """{kernel: {counter: [value per dispatch]}} of one pass."""
        out = {}
        for r in _csv_rows(os.path.join(d, sub)):
            k = _kernel_key(r.get("Kernel_Name", ""))
            if k:
                out.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        return out

    def read_bytes(pas, k):
        c = pas.get(k, {})
        if not all(n in c for n in RDREQ):
            return None
        return statistics.median([32 * a + 64 * b + 128 * e for a, b, e in zip(*(c[n] for n in RDREQ))])

    def med(pas, k, name, scale=1.0):
        c = pas.get(k, {})
        return statistics.median(c[name]) * scale if name in c else None

    rd, wr, fe = per_dispatch("rdreq"), per_dispatch("write"), per_dispatch("fetch")
    check = {}
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib * (1 << 20)
        crd, cwr, cfe = per_dispatch("crdreq"), per_dispatch("cwrite"), per_dispatch("cfetch")
        check = {"copy_bytes": nbytes,
                 "read_by_request_size_over_copy": (read_bytes(crd, "copyBuffer") or float("nan")) / nbytes,
                 "write_size_over_copy": (med(cwr, "copyBuffer", "WRITE_SIZE", 1024) or float("nan")) / nbytes,
                 "fetch_size_over_copy": (med(cfe, "copyBuffer", "FETCH_SIZE", 1024) or float("nan")) / nbytes}
    dom = max((k for k in stats if k.startswith("k_") and not k.startswith("k_spec")),
              key=lambda k: sum(stats[k]))
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    lines = [f"# Kernel durations and HBM traffic: {w}, FP32-mixed form", "",
             f"Command: `{args.profile_command}`", "",
             "| kernel | launches | avg ms | total ms |", "|---|---|---|---|"]
    for k, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| {k} | {len(v)} | {statistics.mean(v):.4f} | {sum(v):.3f} |")
    lines += ["", "HBM traffic per launch: reads = 32/64/128-byte L2-to-memory read requests "
              "(TCC_EA0_RDREQ_32B/64B/128B) times their sizes, writes = WRITE_SIZE; FETCH_SIZE "
              "(which counts 128-byte requests from TCC_BUBBLE) beside the reads for comparison; "
              "algorithmic bytes = what the method must move:", "",
              "| kernel | read MB | FETCH_SIZE MB | write MB | algorithmic MB |", "|---|---|---|---|---|"]
    ab = algorithmic_bytes(dict(__import__("paper_1804_07135_amd.inputs", fromlist=["WORKLOADS"]).WORKLOADS[w]), 4)
    per_kernel = {}
    for k in sorted(stats, key=lambda k: -sum(stats[k])):
        r_, w_, f_ = read_bytes(rd, k), med(wr, k, "WRITE_SIZE", 1024), med(fe, k, "FETCH_SIZE", 1024)
        if r_ is not None and w_ is not None:
            per_kernel[k] = {"read_bytes": r_, "write_bytes": w_, "avg_ms": statistics.mean(stats[k])}
            if f_ is not None:
                per_kernel[k]["fetch_size_bytes"] = f_
        lines.append(f"| {k} | {(r_ or float('nan')) / 1e6:.1f} | {(f_ or float('nan')) / 1e6:.1f} | "
                     f"{(w_ or float('nan')) / 1e6:.1f} | {(ab[k] / 1e6) if k in ab else float('nan'):.1f} |")
    if check:
        lines += ["", f"Counter check on a {args.copy_probe_mib} MiB device copy: reads by request size "
                  f"{check['read_by_request_size_over_copy']:.4f} x the copied bytes, WRITE_SIZE "
                  f"{check['write_size_over_copy']:.4f} x, FETCH_SIZE {check['fetch_size_over_copy']:.4f} x."]
    # instruction and stall counters, when those passes were collected
    sq = {}
    for sub in ("sqa", "sqb"):
        for k, cs in per_dispatch(sub).items():
            for c, v in cs.items():
                sq.setdefault(k, {})[c] = v
    if sq:
        names = sorted({c for v in sq.values() for c in v})
        lines += ["", "SQ counters per launch (medians; instruction counts are per wavefront):", "",
                  "| kernel | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
        for k in sorted(sq, key=lambda k: -sum(stats.get(k, [0]))):
            if k.startswith("k_") and not k.startswith("k_spec"):
                lines.append(f"| {k} | " + " | ".join(
                    f"{statistics.median(sq[k][c]):.3g}" if c in sq[k] else "" for c in names) + " |")
        for k in per_kernel:
            if k in sq and "SQ_INSTS_VALU" in sq[k]:
                per_kernel[k]["valu_wave_instructions"] = statistics.median(sq[k]["SQ_INSTS_VALU"])
            if k in sq and all(c in sq[k] for c in ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32",
                                                    "SQ_INSTS_VALU_MUL_F32")):
                # executed FP32 flops: 64 lanes per wave instruction, 2 per FMA
                m = {c: statistics.median(sq[k][c]) for c in sq[k]}
                per_kernel[k]["fp32_flops"] = 64 * (2 * m["SQ_INSTS_VALU_FMA_F32"] + m["SQ_INSTS_VALU_ADD_F32"]
                                                    + m["SQ_INSTS_VALU_MUL_F32"])
    lines.append("")
    with open(os.path.join(ROOT, "profiles", f"kernels_{w}_fp32.md"), "w") as fh:
        fh.write("\n".join(lines))
    dk = per_kernel.get(dom, {})
    with open(os.path.join(ROOT, "profiles", f"traffic_{dom}_{w}_fp32.json"), "w") as fh:
        json.dump({"kernel": dom, "workload": w,
                   "bytes_per_launch": dk.get("read_bytes", 0) + dk.get("write_bytes", 0),
                   "read_bytes": dk.get("read_bytes"), "write_bytes": dk.get("write_bytes"),
                   "counter_check": check, "kernels": per_kernel,
                   "kernel_source_hash": kernel_source_hash(), "command": args.profile_command}, fh, indent=1)
    print(json.dumps({"dominant": dom, "read_MB": (dk.get("read_bytes") or 0) / 1e6,
                      "write_MB": (dk.get("write_bytes") or 0) / 1e6, "check": check}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tube_256x256x8_k48")
    ap.add_argument("--graph-chunk", type=int, default=10)
    ap.add_argument("--fp64-steps", type=int, default=0, help="steps of the FP64 plain run (0: = --steps)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="skip the FP64 plain run (profiling)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--rk-iters", type=int, default=5,
                    help="string iterations of the adaptive Dormand-Prince leg (0: skip)")
    ap.add_argument("--rk-interval", type=float, default=0.5)
    ap.add_argument("--paper-steps", type=int, default=200,
                    help="timed iterations of the paper-shape leg (0: skip)")
    ap.add_argument("--paper-batch", type=int, default=16,
                    help="(d, k) points of the batched paper-shape run")
    ap.add_argument("--rk-tol", type=float, default=1e-5)
    ap.add_argument("--full-run-iters", type=int, default=500,
                    help="iterations of the full-run barrier comparison of both forms (0: skip)")
    ap.add_argument("--sweep-iters", type=int, default=20000,
                    help="iteration cap of the 64-point sweep leg (0: skip)")
    ap.add_argument("--sweep-tol", type=float, default=1e-4)
    ap.add_argument("--config-steps", type=int, default=200,
                    help="timed iterations of the small-workload rates (0: skip)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the FP32 form's tiles with the library's autotuner before timing")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--summarize-profiles", default="",
                    help="directory of rocprofv3 CSV outputs (trace/, rdreq/, write/, fetch/, sqa/, sqb/ and the "
                         "copy probe's crdreq/, cwrite/, cfetch/): write the kernel and traffic summaries into "
                         "profiles/ and exit")
    ap.add_argument("--profile-command", default="", help="command line recorded in the summaries")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the method is built and "
              "measured on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1804_07135_amd import inputs, ssm

    if args.copy_probe_mib:
        # known-size copy: reads and writes exactly copy_probe_mib MiB per launch
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}), flush=True)
        return

    w = dict(inputs.WORKLOADS[args.workload])
    prob = dict(nx=w["nx"], ny=w["ny"], nz=w["nz"], K=w["K"], J=w["J"], d=w["d"], ku=w["ku"], D=w["D"])
    s0 = inputs.build_string(w)
    KN = w["K"] * w["nx"] * w["ny"] * w["nz"]
    tau = w["tau"]
    steps, warm = args.steps, args.warmup

    # --- FP32-mixed form, graph replay -------------------------------------
    gchunk = replay_chunk(warm, args.graph_chunk)
    sm = ssm.StringMethod(prob, ssm.SSM_FP32_MIXED)
    sm.set_options(check_every=10, graph_chunk=gchunk)
    sm.set_string(s0)
    tiles = None
    if args.autotune:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            cache = os.path.join(td, "tiles.txt")
            sm.autotune(cache)
            with open(cache) as fh:
                tiles = fh.read().strip()
        sm.set_string(s0)
    sm.iterate(warm, tau)
    dt32 = time_iterations(sm, steps, tau)
    bar32 = sm.barrier().cpu().numpy()[0]
    flags = sm.check()
    # per-kernel durations with HIP events on the library's stream, same steps
    sm.profile(True)
    sm.profile_read()
    dt32_ev = time_iterations(sm, steps, tau)
    prof = sm.profile_read()
    sm.profile(False)
    # field of the initial string (rounded to FP32) in this form, for the
    # normwise field error against the FP64 form on the same spins
    s0_32 = s0.astype(np.float32)
    _, h32, _ = sm.eval(spins=s0_32, want_field=True, want_terms=False)
    del sm
    torch.cuda.empty_cache()

    # --- FP64 plain form, direct launches ----------------------------------
    st64 = args.fp64_steps or steps
    if args.fp32_only:
        print(json.dumps({"ms_per_step": dt32 / steps * 1e3, "kernels_ms": prof, "tiles": tiles}), flush=True)
        return
    sm64 = ssm.StringMethod(prob, ssm.SSM_FP64)
    _, h64, _ = sm64.eval(spins=s0_32.astype(np.float64), want_field=True, want_terms=False)
    hd = (h32.double() - h64).reshape(w["K"], -1)
    field_err = float((hd.norm(dim=1) / h64.reshape(w["K"], -1).norm(dim=1)).max())
    del h32, h64, hd
    sm64.set_string(s0)
    sm64.iterate(warm, tau)
    dt64 = time_iterations(sm64, st64, tau)
    bar64 = sm64.barrier().cpu().numpy()[0]
    del sm64
    torch.cuda.empty_cache()

    # barrier of both forms after the same number of iterations (warm + steps)
    same_iters = (st64 == steps)
    bar_err = float(abs(bar32[0] - bar64[0]) / max(abs(bar64[0]), 1e-300)) if same_iters else None

    value = steps * KN / dt32
    value64 = st64 * KN / dt64
    # dominant kernel (and the runner-up) and their rooflines
    ab = algorithmic_bytes(w, 4)
    kern = {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / max(v[1], 1)} for k, v in prof.items()}
    ranked = sorted((k for k in kern if k in ab), key=lambda k: -kern[k]["ms_total"])
    dom = ranked[0]
    # per-kernel measured traffic and instruction counts from the committed
    # rocprofv3 summary, used only while it covers the same kernel sources
    pk = {}
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if name.startswith("traffic_") and name.endswith(f"_{args.workload}_fp32.json"):
            with open(os.path.join(ROOT, "profiles", name)) as fh:
                tr = json.load(fh)
            if tr.get("kernel_source_hash") == kernel_source_hash():
                pk = tr.get("kernels", {})
    floor_bytes = 72 * KN  # read/write floor of one fused FP32 iteration

    def roofline_of(k):
        """HBM roofline of kernel k: algorithmic bytes per launch over its
        average launch duration (HIP events on the launch stream)."""
        t_avg = kern[k]["ms_avg"] * 1e-3
        traffic = (pk[k]["read_bytes"] + pk[k]["write_bytes"]) if k in pk else None
        achieved = ab[k] / t_avg / 1e9
        r = {"bound": "hbm", "kernel": k, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": ab[k],
             "avg_launch_ms": kern[k]["ms_avg"],
             "traffic_frac": traffic / t_avg / 1e9 / HBM_PEAK_GBS if traffic else None}
        q = pk.get(k, {})
        if "valu_wave_instructions" in q:
            # a wave64 FP32/FP64 VALU instruction occupies one SIMD for 4
            # cycles; 1024 SIMDs at 2.4 GHz
            r["valu_issue_frac"] = q["valu_wave_instructions"] * 4 / (1024 * 2.4e9 * t_avg)
        if "fp32_flops" in q:
            # the vector-ALU view: FP32 flops the kernel executes (counters:
            # 64 lanes x (2 FMA + ADD + MUL) per wave instruction) against
            # the non-packed FP32 ceiling
            tf = q["fp32_flops"] / t_avg / 1e12
            r["alu_view"] = {"executed_flops_per_launch": q["fp32_flops"], "achieved": tf,
                             "peak": FP32_VECTOR_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                             "frac": tf / FP32_VECTOR_NONPACKED_TFLOPS}
        return r

    roofline = roofline_of(dom)
    roofline_second = roofline_of(ranked[1]) if len(ranked) > 1 else None
    iteration = None
    it_kernels = ("k_xfwd", "k_conv", "k_xinv", "k_arc", "k_reduce", "k_interp")
    if all(k in pk for k in it_kernels):
        # measured HBM bytes of one iteration (counter traffic, redundant
        # re-reads included): every kernel of the iteration once, over the
        # timed iteration (graph replay)
        b = sum(pk[k]["read_bytes"] + pk[k]["write_bytes"] for k in it_kernels)
        rate = b / (dt32 / steps) / 1e9
        iteration = {"measured_bytes_incl_redundant": b, "GBps": rate, "frac": rate / HBM_PEAK_GBS,
                     "floor_bytes": floor_bytes}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-field evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": dt32 / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": [w["nx"], w["ny"], w["nz"]], "images": w["K"],
                   "params": {"J": w["J"], "d": w["d"], "ku": w["ku"], "dip": w["D"]}, "tau": tau,
                   "form": "FP32 spins/FFT/field storage, FP64 per-site arithmetic, energies, arc lengths "
                           "and barrier; " + ("iterations replayed as a HIP graph of %d" % gchunk
                                             if gchunk else "direct launches")},
        "string_iters_per_s": steps / dt32,
        "fp64_plain": {"value": value64, "unit": "site-field evals/s", "steps": st64,
                       "ms_per_step": dt64 / st64 * 1e3, "string_iters_per_s": st64 / dt64},
        "speedup_fp32_batched_vs_fp64_plain": value / value64,
        "barrier_fp32": float(bar32[0]),
        "barrier_fp64": float(bar64[0]),
        "barrier_rel_err_fp32_vs_fp64": bar_err,
        "field_rel_err_fp32_vs_fp64": field_err,
        "failure_flags": int(flags),
        "roofline": roofline,
        "roofline_second": roofline_second,
        "iteration_floor_frac": floor_bytes / (dt32 / steps) / 1e9 / HBM_PEAK_GBS,
        "iteration_traffic": iteration,
        "kernels_ms_avg": {k: round(v["ms_avg"], 5) for k, v in kern.items()},
        "autotuned_tiles": tiles,
        "ms_per_step_with_events": dt32_ev / steps * 1e3,
    }
    if args.full_run_iters > 0:
        out["full_run"] = full_run_leg(ssm, torch, prob, s0, args.full_run_iters, tau, args.graph_chunk)
    if args.config_steps > 0:
        out["small_workloads"] = small_workloads_leg(ssm, torch, inputs, args.config_steps, args.graph_chunk)
    if args.sweep_iters > 0:
        out["sweep_64_points"] = sweep_leg(ssm, torch, inputs, args)
    if args.paper_steps > 0:
        out["paper_shape_112x112x1_k60"] = paper_shape_leg(ssm, torch, args)
    if args.rk_iters > 0:
        out["rk_dopri54"] = rk_leg(ssm, torch, prob, s0, KN, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, s0, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
