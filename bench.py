"""Benchmark: shifted pipelined CG on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (one step): a complete shifted p-CG solve (Alg. 3) of the 3-D
Poisson 7-point problem on a 256^3 grid (16,777,216 unknowns), Jacobi
preconditioner, sigma = 1 (midpoint of spec(A M^-1)), binary64, x_true ~
U(-1, 1) from seed 0, b = A x_true, x0 = 0, to ||r||/||b|| <= 1e-10 with the
explicit-residual check (cap 5000).  A step includes the init passes, every
fused iteration pass, the explicit residual and any restart; inputs are
resident in HBM before the timed region.

Printed: one JSON line with the metric (iterations per second over the K
timed solves), the roofline of the fused iteration pass (algorithmic bytes
per pass / average pass duration from HIP events on the solver's stream, vs
8 TB/s), and the oracle's rate on a bounded sample of the same workload on
the host cores.
"""
from __future__ import annotations

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

METRIC = "shifted p-CG iters/s + HBM GB/s (3D Poisson 256^3); batched solves/s, p99"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pipe_3d7_jacobi_fp64_256.json")
# the rocprofv3 runs whose output --ingest-profile summarises (run from the repo root)
PROFILE_COMMANDS = [
    "rocprofv3 --kernel-trace --stats -d gpurun_out/prof_trace -o trace --output-format csv -- "
    "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-batched --no-serving --no-methods",
    "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_fetch -o fetch --output-format csv -- "
    "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-batched --no-serving --no-methods --max-iter 24 --calib-copy",
    "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_write -o write --output-format csv -- "
    "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-batched --no-serving --no-methods --max-iter 24 --calib-copy",
    "python3 bench.py --ingest-profile gpurun_out/prof_trace gpurun_out/prof_fetch gpurun_out/prof_write",
]
KERNEL_SOURCES = ["paper_1706_05988_amd/csrc/pcg_kernels.h", "paper_1706_05988_amd/csrc/pcg_device.h"]


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code with comments and blank space
    removed: a profile stays valid across comment-only edits."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def bytes_per_unknown(method: str, jacobi: bool, fp32: bool) -> int:
    """Algorithmic HBM bytes per unknown per iteration pass: every stored
    vector read once and written once, w read once (halo counted once) and
    written once into the other buffer; x and b stay binary64.  The fused
    pipelined pass reads and writes x every other iteration (8 bytes per
    iteration on average), classic CG every iteration."""
    es = 4 if fp32 else 8
    if method == "cg":  # per iteration over both passes: r, p(x2), s + x
        return 8 * 2 + es * 8
    if jacobi:  # x rw / 2; r u z q s t p rw; w r, w' w
        return 8 + es * (7 * 2 + 2)
    return 8 + es * (4 * 2 + 2)  # x rw / 2; r z s t rw; w r, w' w


def traffic_entry():
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(p, iters: int) -> dict:
    """The oracle, as it stands, on a bounded sample of the same workload:
    `iters` p-CG-sh iterations (plus its init and final explicit residual)."""
    import oracle
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    r = oracle.solve(p.op, p.b, p.x0, method="pipe_shift", sigma=p.sigma, rtol=1e-30, max_iter=iters,
                     jacobi=True, record=False, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": r["iterations"] / dt, "unit": "iterations/s", "cores": threads, "kind": "oracle",
            "sample": f"{r['iterations']} shifted p-CG iterations of the same 256^3 Jacobi problem "
                      f"(timing includes the oracle's init and final explicit residual), {dt:.1f} s"}


def copy_probe(torch, dev, nbytes: int = 1 << 31, reps: int = 5) -> float:
    """Bytes read plus bytes written per second (GB/s) of torch's device copy
    of `nbytes` into another buffer, averaged over `reps` copies timed with
    events on the current stream, after one untimed copy."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / sec / 1e9


def stream_ceiling(P, torch, n: int = 1 << 24, reps: int = 20) -> dict:
    """Streaming bandwidth of plain probe kernels (pcg_stream_probe, the
    fused passes' tiling) over buffers the size of the headline pass's
    vectors (n values each): read only, copy, and 9 read + 9 written
    binary64 streams -- the fused p-CG-sh pass with Jacobi moves 8.5 + 8.5
    vectors per iteration (x every other iteration), the 9 + 8 mix its
    catch-up pass -- and 8 + 8 binary32 streams (the FP32-stream passes'
    balance of reads and writes); each the fastest of 1, 2 and 4 blocks per
    CU.  GB/s = bytes moved / average launch time."""
    mixes = [("read", 16, 0, n, 0), ("copy", 1, 1, 9 * n, 0), ("r9w8", 9, 8, n, 0), ("r9w9", 9, 9, n, 0),
             ("f32_r8w8", 8, 8, n, P.PCG_PROBE_FP32)]
    need = max(P.stream_probe_bytes(i, o, m) for _, i, o, m, _ in mixes)
    buf = torch.zeros(need + 256, dtype=torch.uint8, device="cuda")
    ptr = (buf.data_ptr() + 255) & ~255
    st = torch.cuda.current_stream().cuda_stream
    out = {"vector_bytes": 8 * n}
    for name, nin, nout, m, f32 in mixes:
        for flags in (0, P.PCG_PROBE_NT, P.PCG_PROBE_NT | P.PCG_PROBE_BLOCKED, P.PCG_PROBE_NT | P.PCG_PROBE_WIDE):
            if name == "copy" and flags & P.PCG_PROBE_BLOCKED:
                continue
            # the persistent grid at 1, 2 and 4 blocks per CU; the fastest counts
            best = 0.0
            for per_cu in (1, 2, 4):
                us = P.pcg_stream_probe(nin, nout, flags | f32 | (per_cu << 8), m, ptr, need, reps, st)
                best = max(best, (nin + nout) * (4 if f32 else 8) * m / (us * 1e-6) / 1e9)
            tag = (("_nt" if flags & P.PCG_PROBE_NT else "") + ("_blocked" if flags & P.PCG_PROBE_BLOCKED else "")
                   + ("_wide" if flags & P.PCG_PROBE_WIDE else ""))
            out[f"{name}{tag}_gbs"] = best
    del buf
    torch.cuda.empty_cache()
    out["best_read_write_gbs"] = max(v for k, v in out.items() if k.startswith(("copy", "r9")))
    out["best_fp32_read_write_gbs"] = max(v for k, v in out.items() if k.startswith("f32_"))
    return out


def _csv(path_glob):
    import csv
    import glob
    files = sorted(glob.glob(path_glob, recursive=True))
    if not files:
        raise FileNotFoundError(path_glob)
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def ingest_profiles(trace_dir: str, fetch_dir: str, write_dir: str, kernel: str, name: str, commands: list):
    """Summarise rocprofv3 output of this benchmark into profiles/:
    the kernel's duration statistics (--kernel-trace --stats) and its HBM
    traffic per launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each
    scaled by what the same counter reads for the 1 GiB device copy that the
    --calib-copy run performs first.  Working passes are the dispatches whose
    value is above half the maximum (passes after convergence return early)."""
    GiB_KiB = 2 ** 20
    stats = _csv(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    trace = _csv(os.path.join(trace_dir, "**", "*kernel_trace.csv"))
    krow = [r for r in stats if kernel in r["Name"]]
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace if kernel in r["Kernel_Name"]]
    work = [d for d in durs if d > 0.5 * max(durs)]
    out = {"kernel": kernel, "kernel_source_hash": kernel_source_hash(), "commands": commands}
    out["rocprof_calls"] = int(krow[0]["Calls"]) if krow else len(durs)
    out["rocprof_average_ns_all"] = float(krow[0]["AverageNs"]) if krow else sum(durs) / len(durs)
    out["working_passes"] = len(work)
    out["average_ns_working"] = sum(work) / len(work)
    ws = sorted(work)
    lo, hi = sum(ws[: len(ws) // 2]) / max(1, len(ws) // 2), sum(ws[len(ws) // 2:]) / max(1, len(ws) - len(ws) // 2)
    out.update(average_ns_fast_half=lo, average_ns_slow_half=hi)

    def counter(dirname, cname):
        rows = _csv(os.path.join(dirname, "**", "*counter_collection.csv"))
        copy = [float(r["Counter_Value"]) for r in rows
                if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == cname]
        kv = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"] and r["Counter_Name"] == cname]
        kv = [v for v in kv if v > 0.5 * max(kv)]
        calib = max(copy)  # the 1 GiB device-to-device copies
        return sum(kv) / len(kv), calib, GiB_KiB / calib

    f_kib, f_cal, f_scale = counter(fetch_dir, "FETCH_SIZE")
    w_kib, w_cal, w_scale = counter(write_dir, "WRITE_SIZE")
    out.update(fetch_kib_per_launch=f_kib, write_kib_per_launch=w_kib,
               copy_1GiB_fetch_kib=f_cal, copy_1GiB_write_kib=w_cal,
               fetch_scale=f_scale, write_scale=w_scale,
               bytes_per_launch=(f_kib * f_scale + w_kib * w_scale) * 1024)
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"traffic_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    top = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:8]
    lines = [f"# rocprofv3 summary: {kernel} ({name})", "",
             "Commands (from the repository root, on the MI355X):", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", "## Kernel statistics (--kernel-trace --stats)", "",
              "| kernel | calls | average ns | % |", "|---|---|---|---|"]
    lines += [f"| {r['Name'][:70]} | {r['Calls']} | {float(r['AverageNs']):.0f} | {float(r['Percentage']):.2f} |"
              for r in top]
    bpp = bytes_per_unknown("pipe_shift", True, False) * 256 ** 3
    lines += ["", f"Working passes of the fused kernel: {len(work)}, average {out['average_ns_working']:.0f} ns "
              f"(all {out['rocprof_calls']} dispatches incl. early-returning ones after convergence: "
              f"{out['rocprof_average_ns_all']:.0f} ns).",
              "Passes alternate between skipping x and catching x up: the faster and slower halves of the "
              f"working passes average {lo:.0f} ns and {hi:.0f} ns.",
              f"Algorithmic bytes per pass: {bpp} -> {bpp / out['average_ns_working']:.0f} GB/s "
              f"({bpp / out['average_ns_working'] / HBM_PEAK_GBS * 100:.1f}% of 8 TB/s).", "",
              "## HBM traffic (--pmc FETCH_SIZE, --pmc WRITE_SIZE; KiB per dispatch)", "",
              f"- calibration: a 1 GiB device copy reads as FETCH_SIZE {f_cal:.0f} KiB and WRITE_SIZE {w_cal:.0f} KiB "
              f"-> scale factors {f_scale:.4f} (fetch), {w_scale:.4f} (write)",
              f"- fused pass: FETCH_SIZE {f_kib:.0f} KiB, WRITE_SIZE {w_kib:.0f} KiB per working dispatch",
              f"- scaled traffic per pass: {out['bytes_per_launch']:.4g} B "
              f"(algorithmic {bpp:.4g} B, ratio {out['bytes_per_launch'] / bpp:.4f})",
              f"- kernel source hash: {out['kernel_source_hash']}", ""]
    with open(os.path.join(ROOT, "profiles", f"{name}.md"), "w") as f:
        f.write("\n".join(lines))
    return out


# Passes profiled one at a time (--profile-pass NAME, then --ingest-pass NAME):
# the workload, the kernel-name prefix rocprofv3 reports, and the storage form.
PASS_PROFILES = {
    "pipe_3d7_jacobi_fp32_256": dict(problem="poisson3d", N=256, fp32=True, kernel="k_pipe<float, 1, true"),
    "pipe_csr_aniso1024_jacobi_fp64": dict(problem="aniso", N=1024, fp32=False, kernel="k_pipe<double, 2, true"),
    "pipe_csr_aniso1024_jacobi_fp32": dict(problem="aniso", N=1024, fp32=True, kernel="k_pipe<float, 2, true"),
    "batch_rect512_fp32_fullpass": dict(problem="batch", N=512, fp32=True, kernel="k_batch_step<float"),
    # banded random CSR (rows of 4..40 entries) on the sorted sliced-ELL copy
    # (the built-in choice there); bytes are the CSR form's, padding excluded
    "pipe_csr_banded4m_jacobi_fp64": dict(problem="banded", N=4_000_000, fp32=False,
                                          kernel="k_pipe<double, 2, true, 4, true, false, 2>"),
    # classic CG's two passes (bytes per unknown: A reads r and p, writes p' and s;
    # B reads x, r, p', s and writes x and r)
    "cg_a_3d7_jacobi_fp64_256": dict(problem="poisson3d", N=256, fp32=False, method="cg",
                                     kernel="k_cg_a_zm<double", bytes_per_unknown=32),
    "cg_b_3d7_jacobi_fp64_256": dict(problem="poisson3d", N=256, fp32=False, method="cg",
                                     kernel="k_cg_b<double, 1, true", bytes_per_unknown=48),
}


def pass_commands(name: str) -> list:
    d = f"gpurun_out/prof_{name}"
    return [
        f"rocprofv3 --kernel-trace --stats -d {d}_trace -o trace --output-format csv -- "
        f"python3 bench.py --profile-pass {name} --passes 200",
        f"rocprofv3 --pmc FETCH_SIZE -d {d}_fetch -o fetch --output-format csv -- "
        f"python3 bench.py --profile-pass {name} --passes 24 --calib-copy",
        f"rocprofv3 --pmc WRITE_SIZE -d {d}_write -o write --output-format csv -- "
        f"python3 bench.py --profile-pass {name} --passes 24 --calib-copy",
        f"python3 bench.py --ingest-pass {name} {d}_trace {d}_fetch {d}_write",
    ]


def pass_workload(name: str, seed: int = 0):
    """(description, algorithmic bytes per working pass, builder) of a
    profiled pass; the builder returns a callable that runs `passes` passes."""
    import problems
    cfg = PASS_PROFILES[name]
    es = 4 if cfg["fp32"] else 8
    if cfg["problem"] == "poisson3d":
        p = problems.poisson3d(cfg["N"], seed=seed)
        n = p.op.n
        if cfg.get("method") == "cg":
            return (f"3-D Poisson 7-point {cfg['N']}^3 (n={n}), Jacobi, classic CG, FP64",
                    cfg["bytes_per_unknown"] * n, p)
        return (f"3-D Poisson 7-point {cfg['N']}^3 (n={n}), Jacobi, p-CG-sh sigma = 1, "
                f"{'FP32-stream' if cfg['fp32'] else 'FP64'}",
                bytes_per_unknown("pipe_shift", True, cfg["fp32"]) * n, p)
    if cfg["problem"] in ("aniso", "banded"):
        if cfg["problem"] == "aniso":
            p = problems.anisotropic_csr(cfg["N"], seed=seed)
            what = f"2-D anisotropic diffusion {cfg['N']}^2 CSR"
        else:
            p = problems.banded_csr(cfg["N"], seed=1)
            what = "banded random CSR, rows of 4..40 entries, sorted sliced-ELL copy"
        n, nnz = p.op.n, int(p.op.row_ptr[-1])
        # streams: x rw every other pass, 7 vectors rw, w r + w' w; CSR values,
        # indices, row_ptr, Jacobi diagonal
        return (f"{what} (n={n}, nnz={nnz}), Jacobi, p-CG-sh sigma = 1, "
                f"{'FP32-stream' if cfg['fp32'] else 'FP64'}",
                n * (8 + es * 16) + nnz * (4 + es) + 4 * (n + 1) + es * n, p)
    ps = problems.batch_rectangles(cfg["N"], seed=seed)
    tot = sum(q.op.n for q in ps)
    # x rw every other pass (8 B on average) + r, z, s, t rw (8 es) + w r, w' w (2 es)
    return (f"{cfg['N']} 2-D Poisson rectangles (sum n = {tot}), FP32-stream p-CG-sh sigma = 4 + c, "
            f"every system iterating", tot * (8 + es * 10), ps)


def run_pass_profile(P, torch, name: str, passes: int):
    """Run `passes` iteration passes of the named workload twice (a warm-up
    solve and the profiled one) with no stop test."""
    cfg = PASS_PROFILES[name]
    desc, bpp, prob = pass_workload(name)
    if cfg["problem"] == "batch":
        bs = [torch.from_numpy(q.b).cuda() for q in prob]
        xs = [torch.zeros_like(b) for b in bs]
        opts = [P.make_options(method="pipe_shift", fp32=True, sigma=q.sigma, rtol=1e-30, max_iter=passes,
                               true_residual_check=False) for q in prob]
        B = P.Batch([q.op for q in prob], opts)
        for _ in range(2):
            for x in xs:
                x.zero_()
            B.solve(bs, xs)
    else:
        method = cfg.get("method", "pipe_shift")
        opt = P.make_options(method=method, jacobi=True, fp32=cfg["fp32"], sigma=1.0 if method == "pipe_shift" else 0.0,
                             rtol=1e-30, max_iter=passes, true_residual_check=False)
        sv = P.Solver(prob.op, opt)
        b = torch.from_numpy(prob.b).cuda()
        x = torch.zeros_like(b)
        for _ in range(2):
            x.zero_()
            sv.solve(b, x)
        sv.close()
    torch.cuda.synchronize()
    print(f"[bench] profile pass {name}: {desc}, {passes} passes x 2, {bpp} algorithmic bytes per pass",
          flush=True)


def ingest_pass(name: str, trace_dir: str, fetch_dir: str, write_dir: str) -> dict:
    """Summarise the rocprofv3 runs of pass_commands(name) into
    profiles/<name>.md: the pass's duration (working dispatches: above half
    the longest), HBM bytes per dispatch from FETCH_SIZE / WRITE_SIZE scaled
    by the 1 GiB calibration copy, both against the algorithmic bytes."""
    cfg = PASS_PROFILES[name]
    kernel = cfg["kernel"]
    desc, bpp, _ = pass_workload(name)
    GiB_KiB = 2 ** 20
    stats = _csv(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    trace = _csv(os.path.join(trace_dir, "**", "*kernel_trace.csv"))
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace if kernel in r["Kernel_Name"]]
    work = [d for d in durs if d > 0.5 * max(durs)]
    avg = sum(work) / len(work)

    def counter(dirname, cname):
        rows = _csv(os.path.join(dirname, "**", "*counter_collection.csv"))
        copy = [float(r["Counter_Value"]) for r in rows
                if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == cname]
        kv = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"] and r["Counter_Name"] == cname]
        kv = [v for v in kv if v > 0.5 * max(kv)]
        calib = max(copy)
        return sum(kv) / len(kv), calib, GiB_KiB / calib

    f_kib, f_cal, f_scale = counter(fetch_dir, "FETCH_SIZE")
    w_kib, w_cal, w_scale = counter(write_dir, "WRITE_SIZE")
    traffic = (f_kib * f_scale + w_kib * w_scale) * 1024
    out = {"pass": name, "kernel": kernel, "workload": desc, "kernel_source_hash": kernel_source_hash(),
           "commands": pass_commands(name), "working_dispatches": len(work), "average_ns": avg,
           "algorithmic_bytes_per_pass": bpp, "achieved_gbs": bpp / avg, "frac_of_8TBs": bpp / avg / HBM_PEAK_GBS,
           "fetch_kib": f_kib, "write_kib": w_kib, "fetch_scale": f_scale, "write_scale": w_scale,
           "traffic_bytes_per_pass": traffic, "traffic_over_algorithmic": traffic / bpp,
           "traffic_gbs": traffic / avg}
    top = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:8]
    lines = [f"# rocprofv3 summary: {name}", "", f"Workload: {desc}.", "",
             "Commands (from the repository root, on the MI355X):", ""]
    lines += [f"    {c}" for c in out["commands"]]
    lines += ["", "## Kernel statistics of the trace run (--kernel-trace --stats)", "",
              "| kernel | calls | average ns | % |", "|---|---|---|---|"]
    lines += [f"| {r['Name'][:80]} | {r['Calls']} | {float(r['AverageNs']):.0f} | {float(r['Percentage']):.2f} |"
              for r in top]
    lines += ["", "## The pass", "",
              f"- kernel `{kernel}...`: {len(work)} working dispatches, average {avg:.0f} ns",
              f"- algorithmic bytes per pass {bpp} -> {bpp / avg:.0f} GB/s = "
              f"{100 * bpp / avg / HBM_PEAK_GBS:.1f}% of 8 TB/s",
              f"- calibration: a 1 GiB device copy reads as FETCH_SIZE {f_cal:.0f} KiB and WRITE_SIZE {w_cal:.0f} KiB "
              f"-> scale factors {f_scale:.4f} (fetch), {w_scale:.4f} (write)",
              f"- counters per working dispatch: FETCH_SIZE {f_kib:.0f} KiB, WRITE_SIZE {w_kib:.0f} KiB -> "
              f"{traffic:.4g} B of HBM traffic ({traffic / bpp:.3f} x the algorithmic bytes, {traffic / avg:.0f} GB/s)",
              f"- kernel source hash: {out['kernel_source_hash']}", ""]
    with open(os.path.join(ROOT, "profiles", f"{name}.md"), "w") as f:
        f.write("\n".join(lines))
    with open(os.path.join(ROOT, "profiles", f"traffic_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def bench_batched(P, torch, count: int = 512, seed: int = 0) -> dict:
    """The 512-system batch: 2-D rectangles with sides U{32..256}, A = L + c I,
    FP32-stream shifted p-CG to 1e-8 (binary64 explicit check) in one
    persistent pass per iteration, against the same systems solved one after
    another, one launch sequence per system, with plain binary64 CG."""
    import numpy as np
    import problems
    ps = problems.batch_rectangles(count, seed=seed)
    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    xs = [torch.zeros_like(b) for b in bs]
    opts = [P.make_options(method="pipe_shift", fp32=True, sigma=p.sigma, rtol=1e-8, max_iter=20000,
                           replace_max=8) for p in ps]
    B = P.Batch([p.op for p in ps], opts)
    B.solve(bs, xs)  # warm-up (graph capture, first touch)
    # the default launch shape, then the autotuner's (tuning outside the timed region)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.solve(bs, xs)
    torch.cuda.synchronize()
    t_default = time.perf_counter() - t0
    x0s = [torch.zeros_like(b) for b in bs]
    shape = B.tune(bs, x0s, xs)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = B.solve(bs, xs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    its = np.array([r["iterations"] for r in res])
    # comparator: each system alone, binary64 classic CG, solvers created up front
    solvers = [P.Solver(p.op, P.make_options(method="cg", rtol=1e-8, max_iter=20000)) for p in ps]
    ys = [torch.zeros_like(b) for b in bs]
    solvers[0].solve(bs[0], ys[0])
    ys[0].zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [sv.solve(b, y) for sv, b, y in zip(solvers, bs, ys)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for sv in solvers:
        sv.close()
    return {
        "workload": f"{count} 2-D Poisson rectangles (sides U{{32..256}}, A = L + cI, c ~ U(0, 0.1)), "
                    f"sum n = {sum(p.op.n for p in ps)}, FP32-stream shifted p-CG sigma = 4 + c to 1e-8",
        "solves_per_s": count / t_batch,
        "seconds": t_batch,
        "launch_shape": {"grid_blocks": shape["grid_blocks"] or "default", "passes_per_launch":
                         shape["iters_per_launch"] or "default",
                         "tuned_by": "pcg_batch_tune"},
        "default_shape_solves_per_s": count / t_default,
        "converged": int(sum(r["status"] == "converged" for r in res)),
        "max_true_residual": float(max(r["rel_res_true"] for r in res)),
        "iterations_min_median_max": [int(its.min()), int(np.median(its)), int(its.max())],
        "sequential_fp64_cg": {"solves_per_s": count / t_seq, "seconds": t_seq,
                               "max_true_residual": float(max(r["rel_res_true"] for r in seq))},
        "speedup_vs_sequential": t_seq / t_batch,
    }


def bench_methods(P, torch, p, b, repeats: int = 3) -> list:
    """Config 2's comparison on the headline problem (256^3, Jacobi, x0 = 0,
    to 1e-10 with the binary64 explicit check): classic CG and p-CG in
    binary64 and p-CG-sh in the FP32-stream form, each solved `repeats`
    times after one warm-up.  Per method: iterations, iterations/s over the
    timed solves, explicit residual, and the roofline of its iteration
    passes on its own algorithmic bytes (HIP-event time of the iteration
    launches on the solver's stream)."""
    n = p.op.n
    out = []
    for method, fp32 in (("cg", False), ("pipe", False), ("pipe_shift", True)):
        sig = p.sigma if method == "pipe_shift" else 0.0
        opt = P.make_options(method=method, jacobi=True, fp32=fp32, sigma=sig, rtol=1e-10, max_iter=5000,
                             replace_max=8, timing=True)
        sv = P.Solver(p.op, opt)
        x = torch.zeros_like(b)
        sv.solve(b, x)
        torch.cuda.synchronize()
        rs = []
        t0 = time.perf_counter()
        for _ in range(repeats):
            x.zero_()
            rs.append(sv.solve(b, x))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sv.close()
        its = sum(r["iterations"] for r in rs)
        passes = sum(r["iter_passes"] for r in rs)
        kern_s = sum(r["iter_kernel_ms"] for r in rs) * 1e-3
        bpu = bytes_per_unknown(method, True, fp32)
        per_pass = bpu * n / (2 if method == "cg" else 1)
        achieved = per_pass * passes / kern_s / 1e9
        out.append({
            "method": method, "form": "fp32-stream" if fp32 else "fp64", "sigma": sig,
            "status": rs[-1]["status"], "iterations": rs[-1]["iterations"], "restarts": rs[-1]["replacements"],
            "true_residual_max": max(r["rel_res_true"] for r in rs),
            "iterations_per_s": its / wall, "ms_per_solve": wall / repeats * 1e3,
            "roofline": {"bound": "hbm", "bytes_per_unknown": bpu, "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "avg_pass_us": kern_s / passes * 1e6,
                         "kernel": "k_cg_a + k_cg_b" if method == "cg" else "k_pipe"},
        })
        print(f"[bench] {method} {'fp32-stream' if fp32 else 'fp64'}: {rs[-1]['iterations']} it, "
              f"{its / wall:.0f} it/s, true {out[-1]['true_residual_max']:.3e}, {achieved:.0f} GB/s", flush=True)
    return out


def _serving_pool(log10_max: float, seed: int):
    """Operators for the serving stream: sizes on a grid of quarter decades
    from 1e3 to 10^log10_max; per size a 3-D cube (side round(n^(1/3))) and a
    random banded CSR matrix (generated once, shared by the requests that draw
    that size class)."""
    import numpy as np
    import problems
    levels = np.arange(3.0, log10_max + 1e-9, 0.25)
    pool = {}
    for lv in levels:
        n = int(round(10 ** lv))
        side = max(2, int(round(n ** (1.0 / 3.0))))
        pool[(lv, "3d7")] = problems.stencil3d(side)
        pool[(lv, "csr")] = problems.banded_csr(n, seed=seed + int(lv * 100)).op
    return levels, pool


def bench_serving(P, torch, count: int, log10_max: float, seed: int = 0) -> dict:
    """Poisson arrivals of FP32-stream shifted p-CG requests (to 1e-8, binary64
    explicit check): half 3-D cubes with Jacobi, half banded CSR with Jacobi,
    sigma = 1, sizes log-uniform (quantised to quarter decades).  First a
    saturated run (all requests at t = 0) measures capacity; then arrivals at
    0.7 x that rate give p50 / p99 latency (arrival -> result).  Comparator:
    the same requests solved one at a time in arrival order with plain
    binary64 CG, latencies from a FIFO schedule of their measured service
    times (solver creation -- validation and set-up, as the server's
    admission does -- plus the solve) against the same arrival times.
    Operators are resident on the device for both (uploaded once, outside
    the timed runs); right-hand sides arrive with the requests."""
    import numpy as np
    levels, pool = _serving_pool(log10_max, seed)
    dev32 = {key: P.DeviceOperator(op, P.PCG_FP32_STREAM) for key, op in pool.items()}
    dev64 = {key: P.DeviceOperator(op, P.PCG_FP64) for key, op in pool.items()}
    rng = np.random.default_rng(seed)
    reqs, keys = [], []
    for k in range(count):
        lv = levels[np.abs(levels - rng.uniform(3.0, log10_max)).argmin()]
        kind = "3d7" if rng.uniform() < 0.5 else "csr"
        keys.append((lv, kind))
        b = torch.from_numpy(rng.uniform(-1.0, 1.0, pool[(lv, kind)].n)).cuda()
        reqs.append((dev32[(lv, kind)], b))
    arena = int(16 << 30)
    shape = {"grid_blocks": 0, "iters_per_launch": 0}

    def opts():
        o = P.make_options(method="pipe_shift", jacobi=True, fp32=True, sigma=1.0, rtol=1e-8,
                           max_iter=20000, replace_max=8)
        o.grid_blocks, o.iters_per_launch = shape["grid_blocks"], shape["iters_per_launch"]
        return o

    # launch shape of the server: pcg_batch_tune on a sample of the request mix
    sample = list(range(min(48, count)))
    tb = P.Batch([reqs[k][0] for k in sample], [opts() for _ in sample])
    x0s = [torch.zeros_like(reqs[k][1]) for k in sample]
    shape.update(tb.tune([reqs[k][1] for k in sample], x0s, [torch.zeros_like(x) for x in x0s]))
    del tb, x0s

    def run(arrivals):
        """Submit at the scheduled arrival times; each result's latency is
        counted from its scheduled arrival (a late submit adds its lateness)."""
        srv = P.Server(arena, max_slots=512)
        xs = [torch.zeros_like(b) for _, b in reqs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets, late = [], []
        for (op, b), x, ta in zip(reqs, xs, arrivals):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            late.append(max(0.0, time.perf_counter() - (t0 + ta)))
            tickets.append(srv.submit(op, opts(), b, x))
        res = [srv.wait(t) for t in tickets]
        total = time.perf_counter() - t0
        info = srv.info()
        srv.close()
        for r, lt in zip(res, late):
            r["latency"] = r["seconds"] + lt
        return res, total, info

    run([0.0] * min(8, count))  # warm-up
    sat, t_sat, _ = run([0.0] * count)
    capacity = count / t_sat
    rate = 0.7 * capacity
    arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
    live, t_live, info = run(list(arrivals))
    lat = [r["latency"] for r in live]
    print(f"[bench] serving: capacity {capacity:.1f} solves/s, live {count / t_live:.1f} solves/s, "
          f"p99 {_pct(lat, 99):.4f} s", flush=True)
    # comparator: one request at a time, binary64 CG, service times measured alone
    service = []
    for key, (_, b) in zip(keys, reqs):
        y = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv = P.Solver(dev64[key], P.make_options(method="cg", jacobi=True, rtol=1e-8, max_iter=20000))
        sv.solve(b, y)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        sv.close()
    done, fifo_lat = 0.0, []
    for ta, sv_t in zip(arrivals, service):
        start = max(done, ta)
        done = start + sv_t
        fifo_lat.append(done - ta)
    sizes = [int(reqs[k][0].struct.n) for k in range(count)]
    return {
        "workload": f"{count} requests, n log-uniform 1e3..1e{log10_max:g} (quarter-decade size classes, "
                    f"largest drawn n = {max(sizes)}), half 3-D 7-point cubes, half banded CSR (7-27 nnz/row), "
                    f"Jacobi, sigma = 1, FP32-stream shifted p-CG to 1e-8; arena {arena >> 30} GiB",
        "requests": count,
        "largest_n": max(sizes),
        "requests_above_1e6": int(sum(n > 10 ** 6 for n in sizes)),
        "capacity_solves_per_s": capacity,
        "launch_shape": {"grid_blocks": shape["grid_blocks"] or "default", "passes_per_launch":
                         shape["iters_per_launch"] or "default",
                         "tuned_by": f"pcg_batch_tune on the first {len(sample)} requests"},
        "arrival_rate_hz": rate,
        "solves_per_s": count / t_live,
        "p50_latency_s": _pct(lat, 50),
        "p99_latency_s": _pct(lat, 99),
        "latency_from": "scheduled arrival",
        "converged": int(sum(r["status"] == "converged" for r in live)),
        "max_true_residual": float(max(r["rel_res_true"] for r in live)),
        "max_resident_requests": info["max_running"],
        "launches": info["launches"],
        "joined_a_running_batch": int(sum(r["admitted_at"] > 0 for r in live)),
        "sequential_fp64_cg": {"solves_per_s": count / sum(service), "p50_latency_s": _pct(fifo_lat, 50),
                               "p99_latency_s": _pct(fifo_lat, 99)},
    }


def lanczos_extremes(alpha, beta):
    """Extreme Ritz values of the CG Lanczos matrix (diagonal 1/alpha_i +
    beta_i/alpha_{i-1}, off-diagonal sqrt(beta_i)/alpha_{i-1}) from an
    alpha / beta history: estimates of the spectrum bounds of A M^-1."""
    import numpy as np
    from scipy.linalg import eigh_tridiagonal
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    k = int(np.argmax(~np.isfinite(a))) if not np.all(np.isfinite(a)) else len(a)
    a, b = a[:k], b[:k]
    d = 1.0 / a
    d[1:] += b[1:] / a[:-1]
    e = np.sqrt(b[1:]) / a[:-1]
    ev = eigh_tridiagonal(d, e, eigvals_only=True)
    return float(ev[0]), float(ev[-1])


def _timed_solve(P, torch, op, opts, b):
    s = P.Solver(op, opts)
    x = torch.zeros_like(b)
    s.solve(b, x)  # warm-up (graph)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve(b, x)
    torch.cuda.synchronize()
    r["wall_s"] = time.perf_counter() - t0
    s.close()
    return r


def report_c3(P, torch, N: int, max_iter: int) -> dict:
    """2-D anisotropic diffusion (CSR), Jacobi: attainable explicit residual
    per storage form and shift sigma in {0, lambda_min estimate, midpoint 1,
    lambda_max bound 2}, running to the iteration cap with no stop; plus the
    iteration rate and effective bandwidth of each form, and solves to 1e-10
    and 1e-13 with the explicit check in both forms (the FP32-stream one
    refined by restarts from the binary64 x)."""
    import problems
    p = problems.anisotropic_csr(N, seed=0)
    b = torch.from_numpy(p.b).cuda()
    # lambda_min of spec(D^-1 A) from the Lanczos values of a CG run
    h = _timed_solve(P, torch, p.op, P.make_options(method="cg", jacobi=True, rtol=1e-10, max_iter=max_iter,
                                                    history_cap=max_iter + 2, true_residual_check=False), b)
    k = h["iterations"]
    lmin, lmax = lanczos_extremes(h["alpha"][:k], h["beta"][:k])
    out = {"workload": f"2-D anisotropic diffusion {N}x{N} CSR (n={p.op.n}, nnz={p.op.nnz}), Jacobi",
           "lanczos_lambda_min": lmin, "lanczos_lambda_max": lmax, "kappa_estimate": lmax / lmin,
           "cg_fp64_iterations_to_1e-10": h["iterations"], "runs": []}
    nnz, n = p.op.nnz, p.op.n
    for fp32 in (False, True):
        es = 4 if fp32 else 8
        # streams: x rw every other iteration (8) + 7 vectors rw + w r/w, CSR values +
        # indices + row_ptr + dinv
        bytes_it = n * (8 + es * 16) + nnz * (4 + es) + 4 * (n + 1) + es * n
        for name, sig in (("0", 0.0), ("lambda_min", lmin), ("mid", 1.0), ("lambda_max_bound", 2.0)):
            r = _timed_solve(P, torch, p.op, P.make_options(method="pipe_shift", jacobi=True, fp32=fp32, sigma=sig,
                                                            rtol=1e-30, max_iter=max_iter,
                                                            true_residual_check=False, timing=True), b)
            out["runs"].append({"form": "fp32-stream" if fp32 else "fp64", "sigma": name, "sigma_value": sig,
                                "status": r["status"], "iterations": r["iterations"],
                                "true_residual": r["rel_res_true"],
                                "iters_per_s": r["iterations"] / r["wall_s"],
                                "gbs_algorithmic": bytes_it * r["iter_passes"] / (r["iter_kernel_ms"] * 1e-3) / 1e9})
    # solves with the binary64 explicit check at sigma = 1: the FP32-stream
    # form restarts from the binary64 x until the explicit residual holds
    # (iterative refinement), against the all-binary64 form
    out["refinement"] = []
    for rtol in (1e-10, 1e-13):
        for fp32 in (False, True):
            r = _timed_solve(P, torch, p.op, P.make_options(method="pipe_shift", jacobi=True, fp32=fp32, sigma=1.0,
                                                            rtol=rtol, max_iter=60000, replace_max=40), b)
            out["refinement"].append({"form": "fp32-stream" if fp32 else "fp64", "rtol": rtol, "status": r["status"],
                                      "iterations": r["iterations"], "restarts": r["replacements"],
                                      "true_residual": r["rel_res_true"], "seconds": r["wall_s"]})
    return out


def report_csr_sizes(P, torch, sizes=(512, 1024, 2048, 4096), passes: int = 200) -> dict:
    """The fused CSR pass (2-D anisotropic diffusion N^2, Jacobi, p-CG-sh
    sigma = 1) over grid sizes, both storage forms, reading the operator as
    CSR or as its sliced-ELL copy, at the built-in launch shape: average
    microseconds per pass (HIP events over `passes` passes) and algorithmic
    GB/s.  A fit t = t0 + bytes / BW over the sizes separates the per-pass
    fixed cost from the streaming rate."""
    import numpy as np
    import problems
    out = {"workload": "2-D anisotropic diffusion N^2 CSR, Jacobi, p-CG-sh sigma = 1, " f"{passes} passes", "runs": []}
    for N in sizes:
        p = problems.anisotropic_csr(N, seed=0)
        n, nnz = p.op.n, p.op.nnz
        b = torch.from_numpy(p.b).cuda()
        for fp32 in (False, True):
            es = 4 if fp32 else 8
            bpp = n * (8 + es * 16) + nnz * (4 + es) + 4 * (n + 1) + es * n
            dev = P.DeviceOperator(p.op, P.PCG_FP32_STREAM if fp32 else P.PCG_FP64)
            for sell in (False, True):
                # the built-in CSR shapes: binary64 1 row per thread, 128 threads;
                # FP32-stream 2 rows per thread, 256 threads; 4 blocks per CU
                var = P.PCG_VAR_SET | P.PCG_VAR_NT | (0 if fp32 else P.PCG_VAR_EPT1) | (P.PCG_VAR_CSR_SELL if sell else 0)
                opt = P.make_options(method="pipe_shift", jacobi=True, fp32=fp32, sigma=1.0, rtol=1e-30,
                                     max_iter=passes, true_residual_check=False, timing=True, variant=var,
                                     block_size=256 if fp32 else 128, grid_blocks=1024)
                sv = P.Solver(dev, opt)
                x = torch.zeros_like(b)
                sv.solve(b, x)
                x.zero_()
                r = sv.solve(b, x)
                sv.close()
                us = r["iter_kernel_ms"] * 1e3 / max(1, r["iter_passes"])
                out["runs"].append({"N": N, "n": n, "nnz": nnz, "form": "fp32-stream" if fp32 else "fp64",
                                    "operand": "sliced-ELL" if sell else "CSR", "us_per_pass": us,
                                    "bytes_per_pass": bpp, "gbs": bpp / (us * 1e-6) / 1e9})
                print(out["runs"][-1], flush=True)
            del dev
        del b
        torch.cuda.empty_cache()
    for form in ("fp64", "fp32-stream"):
        for operand in ("CSR", "sliced-ELL"):
            rs = [r for r in out["runs"] if r["form"] == form and r["operand"] == operand]
            A = np.array([[1.0, r["bytes_per_pass"]] for r in rs])
            t = np.array([r["us_per_pass"] * 1e-6 for r in rs])
            (t0, inv_bw), *_ = np.linalg.lstsq(A, t, rcond=None)
            out[f"fit_{form}_{operand}"] = {"fixed_us": t0 * 1e6, "streaming_gbs": 1.0 / inv_bw / 1e9}
    return out


def report_csr_shapes(P, torch, sizes=(1024, 2048), passes: int = 200) -> dict:
    """Launch shapes of the fused CSR pass (2-D anisotropic diffusion N^2,
    Jacobi, p-CG-sh sigma = 1), both storage forms, CSR rows or the
    sliced-ELL copy: 1, 2 or 4 rows per thread x 128 or 256 threads x 1, 2,
    4 (and for 128 threads 8) blocks per CU; microseconds per pass over
    `passes` passes (HIP events), then the built-in shape for reference."""
    import problems
    out = {"workload": f"2-D anisotropic diffusion N^2 CSR, Jacobi, p-CG-sh sigma = 1, {passes} passes",
           "runs": []}
    ept_bits = {1: P.PCG_VAR_EPT1, 2: 0, 4: P.PCG_VAR_EPT4}
    for N in sizes:
        p = problems.anisotropic_csr(N, seed=0)
        n, nnz = p.op.n, p.op.nnz
        b = torch.from_numpy(p.b).cuda()
        for fp32 in (False, True):
            es = 4 if fp32 else 8
            bpp = n * (8 + es * 16) + nnz * (4 + es) + 4 * (n + 1) + es * n
            dev = P.DeviceOperator(p.op, P.PCG_FP32_STREAM if fp32 else P.PCG_FP64)
            shapes = [(None, None, None, None)]
            for sell in (False, True):
                for ept in (1, 2, 4):
                    for block in (128, 256):
                        for per_cu in (1, 2, 4, 8):
                            if per_cu == 8 and block != 128:
                                continue
                            shapes.append((sell, ept, block, per_cu))
            best = None
            for sell, ept, block, per_cu in shapes:
                if sell is None:
                    kw = {}
                else:
                    kw = dict(variant=P.PCG_VAR_SET | P.PCG_VAR_NT | ept_bits[ept] | (P.PCG_VAR_CSR_SELL if sell else 0),
                              block_size=block, grid_blocks=per_cu * 256)
                opt = P.make_options(method="pipe_shift", jacobi=True, fp32=fp32, sigma=1.0, rtol=1e-30,
                                     max_iter=passes, true_residual_check=False, timing=True, **kw)
                sv = P.Solver(dev, opt)
                x = torch.zeros_like(b)
                sv.solve(b, x)
                x.zero_()
                r = sv.solve(b, x)
                sv.close()
                us = r["iter_kernel_ms"] * 1e3 / max(1, r["iter_passes"])
                row = {"N": N, "form": "fp32-stream" if fp32 else "fp64",
                       "shape": "built-in" if sell is None else
                       f"{'sell' if sell else 'csr'} ept{ept} b{block} x{per_cu}/CU",
                       "us_per_pass": round(us, 2), "gbs": round(bpp / (us * 1e-6) / 1e9)}
                out["runs"].append(row)
                if best is None or us < best["us_per_pass"]:
                    best = row
            out[f"best_{N}_{'fp32' if fp32 else 'fp64'}"] = best
            print(best, [r for r in out["runs"] if r["shape"] == "built-in"][-1], flush=True)
            del dev
        del b
        torch.cuda.empty_cache()
    return out


SORTED_SHAPES = ((128, 2), (128, 4), (128, 6), (128, 8), (256, 2), (256, 3), (256, 4))


def report_csr_banded(P, torch, sizes=(10 ** 6, 4 * 10 ** 6), passes: int = 200,
                      sorted_shapes=SORTED_SHAPES) -> dict:
    """The fused CSR pass on banded random operators (rows of 4 to 40
    entries, the serving mix's CSR half), Jacobi, p-CG-sh sigma = 1, both
    storage forms: the built-in choice, CSR rows at their best shape, and
    the sorted sliced-ELL copy at 4 rows per thread x (threads, blocks per
    CU) of `sorted_shapes`; microseconds per pass over `passes` passes (HIP
    events) with the form, shape and copy size the solver reports."""
    import problems
    out = {"workload": f"banded random CSR (rows 4..40 entries), Jacobi, p-CG-sh sigma = 1, {passes} passes",
           "runs": []}
    for n in sizes:
        p = problems.banded_csr(n, seed=1)
        nnz = int(p.op.row_ptr[-1])
        b = torch.rand(n, dtype=torch.float64, device="cuda") * 2 - 1
        for fp32 in (False, True):
            es = 4 if fp32 else 8
            bpp = n * (8 + es * 16) + nnz * (4 + es) + 4 * (n + 1) + es * n
            dev = P.DeviceOperator(p.op, P.PCG_FP32_STREAM if fp32 else P.PCG_FP64)
            shapes = [("built-in", {})]
            shapes.append(("csr ept1 b256 x4/CU", dict(variant=P.PCG_VAR_SET | P.PCG_VAR_NT | P.PCG_VAR_EPT1,
                                                      block_size=256, grid_blocks=1024)))
            shapes.append(("csr ept2 b256 x2/CU", dict(variant=P.PCG_VAR_SET | P.PCG_VAR_NT, block_size=256,
                                                      grid_blocks=512)))
            for block, per_cu in sorted_shapes:
                shapes.append((f"sorted ept4 b{block} x{per_cu}/CU",
                               dict(variant=P.PCG_VAR_SET | P.PCG_VAR_NT | P.PCG_VAR_EPT4 | P.PCG_VAR_CSR_SELL_SORTED,
                                    block_size=block, grid_blocks=per_cu * 256)))
            for name, kw in shapes:
                opt = P.make_options(method="pipe_shift", jacobi=True, fp32=fp32, sigma=1.0, rtol=1e-30,
                                     max_iter=passes, true_residual_check=False, timing=True, **kw)
                sv = P.Solver(dev, opt)
                x = torch.zeros_like(b)
                sv.solve(b, x)
                x.zero_()
                r = sv.solve(b, x)
                info = sv.info()
                sv.close()
                us = r["iter_kernel_ms"] * 1e3 / max(1, r["iter_passes"])
                row = {"n": n, "form": "fp32-stream" if fp32 else "fp64", "shape": name,
                       "us_per_pass": round(us, 2), "gbs_on_csr_bytes": round(bpp / (us * 1e-6) / 1e9),
                       "operand": info["csr_form_name"], "ept": info["ept"], "block": info["block"],
                       "grid": info["grid"], "copy_entries_per_nnz": round(info["csr_entries"] / nnz, 3)}
                out["runs"].append(row)
                print(row, flush=True)
            del dev
        del b
        torch.cuda.empty_cache()
    return out


def report_pipe_shapes(P, torch, passes: int = 200) -> dict:
    """Launch shapes of the fused p-CG-sh pass without a preconditioner on
    stencils (the Section 5.2 problem 1000^2, a 3300^2 grid and 256^3), both
    storage forms: 1, 2 or 4 unknowns per thread x 128 or 256 threads x 1,
    2, 4 (and for 128 threads 8) blocks per CU; microseconds per pass over
    `passes` passes (HIP events), and the built-in shape."""
    import problems
    out = {"workload": f"p-CG-sh, M = I, {passes} passes", "runs": []}
    ept_bits = {1: P.PCG_VAR_EPT1, 2: 0, 4: P.PCG_VAR_EPT4}
    cases = [("2d 1000^2", problems.stencil2d(1000), 4.0), ("2d 3300^2", problems.stencil2d(3300), 4.0),
             ("3d 256^3", problems.stencil3d(256), 6.0)]
    for name, op, sig in cases:
        b = torch.rand(op.n, dtype=torch.float64, device="cuda") * 2 - 1
        for fp32 in (False, True):
            bpp = op.n * bytes_per_unknown("pipe_shift", False, fp32)
            shapes = [None] + [(e, bl, pc) for e in (1, 2, 4) for bl in (128, 256) for pc in (1, 2, 4, 8)
                               if not (pc == 8 and bl != 128)]
            best = None
            for sh in shapes:
                kw = {} if sh is None else dict(variant=P.PCG_VAR_SET | P.PCG_VAR_NT | ept_bits[sh[0]],
                                                block_size=sh[1], grid_blocks=sh[2] * 256)
                opt = P.make_options(method="pipe_shift", fp32=fp32, sigma=sig, rtol=1e-30, max_iter=passes,
                                     true_residual_check=False, timing=True, **kw)
                sv = P.Solver(op, opt)
                x = torch.zeros_like(b)
                sv.solve(b, x)
                x.zero_()
                r = sv.solve(b, x)
                sv.close()
                us = r["iter_kernel_ms"] * 1e3 / max(1, r["iter_passes"])
                row = {"case": name, "form": "fp32-stream" if fp32 else "fp64",
                       "shape": "built-in" if sh is None else f"ept{sh[0]} b{sh[1]} x{sh[2]}/CU",
                       "us_per_pass": round(us, 2), "gbs": round(bpp / (us * 1e-6) / 1e9)}
                out["runs"].append(row)
                if best is None or us < best["us_per_pass"]:
                    best = row
            print(best, [r for r in out["runs"] if r["shape"] == "built-in"][-1], flush=True)
        del b
        torch.cuda.empty_cache()
    return out


def report_c2(P, torch, N: int = 256) -> dict:
    """The 3-D Poisson problem (N^3, Jacobi, x_true ~ U(-1, 1), x0 = 0):
    classic CG, p-CG and p-CG-sh in binary64, p-CG-sh in the FP32-stream
    form, p-CG with a variable shift (Alg. 4) and p-CG-rr in binary64, each
    to the recursive tolerance 1e-10 with the binary64 explicit check
    (restarts from x until it holds): iterations, time, iterations/s, time
    per iteration, algorithmic GB/s and the fraction of 8 TB/s (p-CG-rr's
    gap-check passes are in its time, not in its bytes), explicit residual.  Then the attainable accuracy of p-CG and p-CG-sh in both forms:
    the explicit residual after 1500 iterations with no stop."""
    import problems
    p = problems.poisson3d(N, seed=0)
    n = p.op.n
    b = torch.from_numpy(p.b).cuda()
    out = {"workload": f"3-D Poisson 7-point {N}^3 (n={n}), Jacobi, x_true ~ U(-1, 1), x0 = 0", "runs": [],
           "attainable_after_1500": []}
    # Alg. 4's schedule here: sigma_{-1} = sigma_0 = 1.5, falling linearly to 1
    # (the spectrum midpoint) at iteration 100 and constant after it
    sched = [1.5] + [1.5 - 0.005 * i for i in range(101)]
    for method, fp32 in (("cg", False), ("pipe", False), ("pipe_shift", False), ("pipe_shift", True),
                         ("pipe_var", False), ("pipe_rr", False)):
        sig = p.sigma if method in ("pipe_shift", "pipe_var") else 0.0
        kw = dict(sigma_schedule=sched) if method == "pipe_var" else {}
        r = _timed_solve(P, torch, p.op, P.make_options(method=method, jacobi=True, fp32=fp32, sigma=sig, rtol=1e-10,
                                                        max_iter=5000, replace_max=8, timing=True, **kw), b)
        its = r["iterations"]
        bytes_it = bytes_per_unknown(method, True, fp32) * n
        kern_s = r["iter_kernel_ms"] * 1e-3
        gbs = bytes_it * its / kern_s / 1e9 if kern_s > 0 else float("nan")
        out["runs"].append({"method": method, "form": "fp32-stream" if fp32 else "fp64",
                            "sigma": "schedule 1.5 -> 1 over 100 iterations" if method == "pipe_var" else sig,
                            "status": r["status"], "iterations": its, "restarts": r["replacements"],
                            "true_residual": r["rel_res_true"], "seconds": r["wall_s"],
                            "iters_per_s": its / r["wall_s"], "us_per_iteration": kern_s * 1e6 / max(1, its),
                            "bytes_per_iteration": bytes_it, "gbs_algorithmic": gbs,
                            "frac_of_8TBs": gbs / HBM_PEAK_GBS})
    for method in ("pipe", "pipe_shift"):
        for fp32 in (False, True):
            sig = p.sigma if method == "pipe_shift" else 0.0
            r = _timed_solve(P, torch, p.op, P.make_options(method=method, jacobi=True, fp32=fp32, sigma=sig,
                                                            rtol=1e-30, max_iter=1500, true_residual_check=False),
                             b)
            out["attainable_after_1500"].append({"method": method, "form": "fp32-stream" if fp32 else "fp64",
                                                 "status": r["status"], "iterations": r["iterations"],
                                                 "true_residual": r["rel_res_true"]})
    return out


def report_small(P, torch) -> dict:
    """Latency-bound cases: 2-D Poisson 100x100 (all three methods, to 1e-12)
    and the 1000x1000 Poisson problem of Section 5.2 (b = A*1, x0 = 0, to
    1e-6 and, as in the accuracy run, 2500 iterations) with CG, p-CG, p-CG-sh
    and p-CG-rr; then the fused pass on a 256 x 256 x 32 grid, one GPU's
    share of the 256^3 problem split into 8 slabs."""
    import problems
    out = {}
    p = problems.poisson2d_manufactured(100)
    b = torch.from_numpy(p.b).cuda()
    for m in ("cg", "pipe", "pipe_shift"):
        r = _timed_solve(P, torch, p.op, P.make_options(method=m, sigma=p.sigma if m == "pipe_shift" else 0.0,
                                                        rtol=1e-12, max_iter=2000, true_residual_check=False,
                                                        timing=True), b)
        out[f"poisson2d_100_{m}"] = {"iterations": r["iterations"], "true_residual": r["rel_res_true"],
                                     "seconds": r["wall_s"], "iters_per_s": r["iterations"] / r["wall_s"],
                                     "us_per_pass": r["iter_kernel_ms"] * 1e3 / max(1, r["iter_passes"])}
    p = problems.paper_parallel_workload(1000)
    b = torch.from_numpy(p.b).cuda()
    for m in ("cg", "pipe", "pipe_shift", "pipe_rr"):
        sig = 4.0 if m == "pipe_shift" else 0.0
        r = _timed_solve(P, torch, p.op, P.make_options(method=m, sigma=sig, rtol=1e-6, max_iter=2500,
                                                        true_residual_check=False), b)
        r2 = _timed_solve(P, torch, p.op, P.make_options(method=m, sigma=sig, rtol=1e-30, max_iter=2500,
                                                         true_residual_check=False), b)
        out[f"paper_poisson2d_1000_{m}"] = {"iterations_to_1e-6": r["iterations"], "seconds_to_1e-6": r["wall_s"],
                                            "replacements_to_1e-6": r["replacements"],
                                            "replacements_long_run": r2["replacements"],
                                            "true_residual_after_2500_or_breakdown": r2["rel_res_true"],
                                            "status_long_run": r2["status"], "iterations_long_run": r2["iterations"],
                                            "seconds_long_run": r2["wall_s"]}
    # one GPU's share of the 256^3 problem split into 8 slabs along z: the
    # fused pass on a 256 x 256 x 32 grid (Jacobi, FP64, p-CG-sh), 400 passes
    p = problems.poisson3d(256, ny=256, nz=32, seed=0)
    op = p.op
    b = torch.from_numpy(p.b).cuda()
    r = _timed_solve(P, torch, op, P.make_options(method="pipe_shift", jacobi=True, sigma=1.0, rtol=1e-300,
                                                  max_iter=400, true_residual_check=False, timing=True), b)
    us = r["iter_kernel_ms"] * 1e3 / max(1, r["iter_passes"])
    out["slab_256x256x32_jacobi_fp64_pipe_shift"] = {
        "unknowns": op.n, "us_per_pass": us, "TB_per_s_on_136B": 136.0 * op.n / (us * 1e-6) / 1e12,
        "iters_per_s": r["iterations"] / r["wall_s"]}
    return out


def report_psi(P, torch) -> dict:
    """Section 5.1 for lapl200: psi_i(sigma) over sigma at i = 500 (the shift
    figure) and psi_i(0), psi_i(sigma*) against i (the right panels of the
    residual-history figure), from alpha / beta recorded on the device by
    500-iteration runs, with the shift picked from them (smallest grid sigma
    within a factor 2 of the smallest psi).  Classic CG's coefficients are
    p-CG's in exact arithmetic and run the full 500 iterations; p-CG's own
    are used when its run is not cut short by a breakdown.  The recursive
    residual histories of p-CG and p-CG-sh at sigma* come along."""
    import numpy as np
    import problems
    p = problems.lapl200()
    b = torch.from_numpy(p.b).cuda()
    runs = {}
    for m in ("pipe", "cg"):
        runs[m] = _timed_solve(P, torch, p.op, P.make_options(method=m, sigma=0.0, rtol=1e-30, max_iter=500,
                                                              history_cap=502, true_residual_check=False), b)
    src = "pipe" if runs["pipe"]["iterations"] == 500 else "cg"
    a, bb = runs[src]["alpha"][:500], runs[src]["beta"][:500]
    i = 499  # psi after 500 iterations (alpha_0 .. alpha_499)
    grid = np.arange(0.0, 8.0001, 0.25)
    t0 = time.perf_counter()
    s_star, vals = P.pcg_select_shift(a, bb, i, grid, slack=2.0)
    its = list(range(10, 500, 10)) + [i]
    psi0 = [P.pcg_psi(a, bb, k, 0.0) for k in its]
    psis = [P.pcg_psi(a, bb, k, s_star) for k in its]
    host_s = time.perf_counter() - t0
    sh = _timed_solve(P, torch, p.op, P.make_options(method="pipe_shift", sigma=s_star, rtol=1e-30, max_iter=500,
                                                     history_cap=502, true_residual_check=False), b)
    return {"problem": "lapl200 (2-D Laplacian 200^2, b = 1/sqrt(n), no preconditioner)",
            "coefficients_from": src, "pipe_iterations": runs["pipe"]["iterations"],
            "pipe_status": runs["pipe"]["status"],
            "fig_shift": {"i": 500, "sigma": grid.tolist(), "psi": vals.tolist(), "sigma_star": s_star,
                          "psi_at_0": float(vals[0]), "psi_at_sigma_star": float(vals[list(grid).index(s_star)]),
                          "paper": {"psi_at_0": 1.78e8, "sigma_star": 4.0, "psi_at_sigma_star": 3.46e2}},
            "fig_history_right": {"i": [k + 1 for k in its], "psi_0": psi0, "psi_sigma_star": psis},
            "recursive_residual": {"pipe": runs["pipe"]["res"][:501].tolist(),
                                   "pipe_shift_sigma_star": sh["res"][:501].tolist()},
            "true_residual_after_500": {"pipe": runs["pipe"]["rel_res_true"], "cg": runs["cg"]["rel_res_true"],
                                        "pipe_shift_sigma_star": sh["rel_res_true"]},
            "host_seconds_for_psi": host_s}


def report_tune(P, torch) -> dict:
    """The autotuner against the built-in launch shapes on the main
    workloads: time per iteration pass (HIP events, 400 timed passes) of
    the default and of the tuned shape."""
    import problems

    def per_pass(op, opts, b):
        o = P.pcg_options.from_buffer_copy(opts)
        o.max_iter, o.rtol, o.true_residual_check, o.timing = 400, 1e-300, 0, 1
        s = P.Solver(op, o)
        x = torch.zeros_like(b)
        s.solve(b, x)
        x.zero_()
        r = s.solve(b, x)
        torch.cuda.synchronize()
        s.close()
        return r["iter_kernel_ms"] * 1e3 / max(1, r["iter_passes"])

    out = {}
    cases = [("3d256_jacobi_fp64_pipe_shift", problems.poisson3d(256, seed=0), dict(jacobi=True, sigma=1.0)),
             ("slab_256x256x32_jacobi_fp64_pipe_shift", problems.poisson3d(256, ny=256, nz=32, seed=0),
              dict(jacobi=True, sigma=1.0)),
             ("3d256_jacobi_fp32_pipe_shift", problems.poisson3d(256, seed=0), dict(jacobi=True, fp32=True, sigma=1.0)),
             ("csr_aniso1024_fp64_pipe_shift", problems.anisotropic_csr(1024, seed=0), dict(jacobi=True, sigma=1.0)),
             ("csr_aniso1024_fp32_pipe_shift", problems.anisotropic_csr(1024, seed=0),
              dict(jacobi=True, fp32=True, sigma=1.0)),
             ("2d1000_fp64_pipe_shift", problems.paper_parallel_workload(1000), dict(sigma=4.0)),
             ("2d1000_fp64_cg", problems.paper_parallel_workload(1000), dict(method="cg"))]
    for name, p, kw in cases:
        kw = dict(kw)
        method = kw.pop("method", "pipe_shift")
        opts = P.make_options(method=method, **kw)
        b = torch.from_numpy(p.b).cuda()
        dev = P.DeviceOperator(p.op, opts.prec)
        t0 = per_pass(dev, opts, b)
        tuned, us = P.tune(dev, opts, b)
        t1 = per_pass(dev, tuned, b)
        out[name] = {"default_us": round(t0, 2), "tuned_us": round(t1, 2), "tuner_us": round(us, 2),
                     "variant": tuned.variant, "block": tuned.block_size, "grid": tuned.grid_blocks}
        print(name, out[name], flush=True)
        del b, dev
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=256, help="grid side (default: the 256^3 workload)")
    ap.add_argument("--fp32", action="store_true", help="FP32-stream form instead of binary64")
    ap.add_argument("--method", default="pipe_shift", choices=["cg", "pipe", "pipe_shift"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=600)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--K", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--max-iter", type=int, default=5000,
                    help="iteration cap (profiling runs use a short fixed count)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-system batch leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--no-methods", action="store_true",
                    help="skip the CG / p-CG / FP32-stream p-CG-sh comparison on the headline problem")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-max-log10", type=float, default=7.0,
                    help="largest request size 10^x (the full range is 7; larger sizes take longer to generate)")
    ap.add_argument("--report", choices=["c2", "c3", "small", "tune", "psi", "batch", "stream", "csr_sizes",
                                         "csr_shapes", "csr_banded", "pipe_shapes"],
                    help="print a measurement report (C3 accuracy per shift, or the latency-bound cases) and exit")
    ap.add_argument("--c3-N", type=int, default=1024)
    ap.add_argument("--c3-max-iter", type=int, default=12000)
    ap.add_argument("--profile-pass", choices=sorted(PASS_PROFILES),
                    help="run a fixed number of passes of one workload (for rocprofv3) and exit")
    ap.add_argument("--passes", type=int, default=200)
    ap.add_argument("--ingest-pass", nargs=4, metavar=("NAME", "TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="summarise the rocprofv3 runs of --profile-pass NAME into profiles/ and exit")
    ap.add_argument("--ingest-profile", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="summarise rocprofv3 output of this benchmark into profiles/ and exit")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (torch) 3 times: the reference kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

    if args.ingest_profile:
        t, fdir, wdir = args.ingest_profile
        res = ingest_profiles(t, fdir, wdir, "k_pipe<double, 1, true", "pipe_3d7_jacobi_fp64_256",
                              commands=PROFILE_COMMANDS)
        print(json.dumps(res, indent=1))
        return

    if args.ingest_pass:
        print(json.dumps(ingest_pass(*args.ingest_pass), indent=1))
        return

    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import problems
    from paper_1706_05988_amd import pcg as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.report:
        rep = (report_c3(P, torch, args.c3_N, args.c3_max_iter) if args.report == "c3" else
               report_small(P, torch) if args.report == "small" else
               report_psi(P, torch) if args.report == "psi" else
               bench_batched(P, torch) if args.report == "batch" else
               stream_ceiling(P, torch) if args.report == "stream" else
               report_csr_sizes(P, torch) if args.report == "csr_sizes" else
               report_csr_shapes(P, torch) if args.report == "csr_shapes" else
               report_csr_banded(P, torch) if args.report == "csr_banded" else
               report_pipe_shapes(P, torch) if args.report == "pipe_shapes" else
               report_c2(P, torch, args.N) if args.report == "c2" else report_tune(P, torch))
        print(json.dumps(rep), flush=True)
        return
    if args.calib_copy:
        src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration: 3 copies of 1 GiB (2^27 doubles) done", flush=True)
        del src, dst
    if args.profile_pass:
        run_pass_profile(P, torch, args.profile_pass, args.passes)
        return
    t_gen = time.perf_counter()
    p = problems.poisson3d(args.N, seed=0, jacobi=True)
    n = p.op.n
    print(f"[bench] generated 3-D Poisson {args.N}^3 (n={n}) in {time.perf_counter() - t_gen:.1f} s", flush=True)
    sigma = p.sigma if args.method == "pipe_shift" else 0.0
    fixed = args.max_iter != 5000
    opt = P.make_options(method=args.method, jacobi=True, fp32=args.fp32, sigma=sigma,
                         rtol=1e-30 if fixed else 1e-10, max_iter=args.max_iter,
                         true_residual_check=not fixed, replace_max=8, timing=True,
                         block_size=args.block, grid_blocks=args.grid, iters_per_launch=args.K,
                         variant=args.variant)
    stream = torch.cuda.current_stream(dev).cuda_stream
    solver = P.Solver(p.op, opt, stream=stream)
    b = torch.from_numpy(p.b).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)

    def step():
        x.zero_()
        return solver.solve(b, x)

    for w in range(args.warmup):
        r = step()
        print(f"[bench] warmup {w}: {r['status']} in {r['iterations']} iterations, "
              f"true residual {r['rel_res_true']:.3e}, {r['seconds']:.3f} s", flush=True)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for k, r in enumerate(results):
        print(f"[bench] step {k}: {r['status']} {r['iterations']} it, true {r['rel_res_true']:.3e}, "
              f"{r['seconds']:.3f} s, pass {r['iter_kernel_ms'] / max(1, r['iter_passes']) * 1e3:.1f} us",
              flush=True)
    iters = sum(r["iterations"] for r in results)
    passes = sum(r["iter_passes"] for r in results)
    kernel_ms = sum(r["iter_kernel_ms"] for r in results)
    bpu = bytes_per_unknown(args.method, True, args.fp32)
    per_pass_bytes = bpu * n / (2 if args.method == "cg" else 1)
    avg_pass_s = kernel_ms / 1e3 / max(1, passes)
    achieved = per_pass_bytes / avg_pass_s / 1e9
    traffic = traffic_entry() if (args.N == 256 and args.method == "pipe_shift" and not args.fp32
                                  and not args.block and not args.grid and not args.variant) else None
    # (not in the counter runs: their calibration takes the largest device copy)
    copy_gbs = None if args.calib_copy else copy_probe(torch, dev)
    out = {
        "metric": METRIC,
        "value": iters / elapsed,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.fp32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3-D Poisson 7-point {args.N}^3 (n={n}), Jacobi, {args.method} "
                        f"sigma={sigma:g}, {'FP32-stream' if args.fp32 else 'FP64'}, full solve to "
                        f"||r||/||b|| <= 1e-10 (explicit-residual check), x0 = 0",
            "n": n,
            "iterations_per_solve": iters / args.steps,
            "true_residual_max": max(r["rel_res_true"] for r in results),
            "hbm_gbs_effective": bpu * n * iters / elapsed / 1e9,
            "algorithmic_bytes_per_iteration": bpu * n,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_pipe (fused p-CG-sh iteration pass)" if args.method != "cg" else "k_cg_a + k_cg_b",
            "avg_pass_us": avg_pass_s * 1e6,
            "bytes_per_pass": per_pass_bytes,
            # the same run's plain device copy (bytes read + written per second):
            # what a kernel with a read / write mix reaches on this HBM
            "copy_probe_gbs": copy_gbs,
        },
        "cpu_baseline": None,
    }
    if args.N == 256 and args.method == "pipe_shift" and not args.fp32 and not fixed:
        # priced as a pass that moves x every iteration (144 B per unknown);
        # this pass moves it every other iteration (136 B on average)
        every = 144 * n / avg_pass_s / 1e9
        out["roofline"]["at_144_bytes_per_unknown"] = {"achieved": every, "frac": every / HBM_PEAK_GBS}
    if not args.calib_copy:
        # plain streaming kernels over the same vector sizes, same run
        sp = stream_ceiling(P, torch, n)
        out["roofline"]["stream_probe"] = sp
        out["roofline"]["frac_of_best_stream_probe"] = achieved / sp["best_read_write_gbs"]
        print(f"[bench] stream probe: read {sp['read_nt_gbs']:.0f}, copy {sp['copy_nt_gbs']:.0f}, "
              f"9r/8w {sp['r9w8_nt_gbs']:.0f} (blocked {sp['r9w8_nt_blocked_gbs']:.0f}), "
              f"9r/9w {sp['r9w9_nt_gbs']:.0f} (blocked {sp['r9w9_nt_blocked_gbs']:.0f}) GB/s (non-temporal)",
              flush=True)
    solver.close()
    del solver, x
    torch.cuda.empty_cache()
    if not args.no_methods and args.N == 256 and not fixed:
        print("[bench] methods leg", flush=True)
        out["methods"] = bench_methods(P, torch, p, b)
    del b
    torch.cuda.empty_cache()
    if not args.no_batched:
        print("[bench] batched leg", flush=True)
        out["batched"] = bench_batched(P, torch)
    if not args.no_serving:
        print("[bench] serving leg", flush=True)
        out["serving"] = bench_serving(P, torch, args.serving_requests, args.serving_max_log10)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", flush=True)
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
