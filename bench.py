"""Benchmark of the batched heat step with FillBoundary on one MI355X.

Workload (default): a 512^3 periodic domain cut by the seeded recursive chop into
~1270 uneven boxes of edge 16..128 (multiples of 8), 5 components, 1 ghost cell,
U(0,1) initial data per component, FP64.  One step = FillBoundary + heat step
over every box and component, run as one launch of the fused kernel; K steps are
one HIP graph.  value = cell updates per second (valid cells x components x K /
timed seconds), in GCell-updates/s.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f64|f32]

Prints one JSON line.  With --gpus above 1 it exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCell-updates/s + % HBM roofline (heat_step+FillBoundary); p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 2 << 30
CPU_SAMPLE_SECONDS = 10.0
CPU_SAMPLE_SECONDS_1T = 5.0   # the one-thread sample of the oracle (at least one step)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "heat_fused_512cube_uneven_5comp_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1604_03570_amd", "csrc", "bl_kernels.hip")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(dtype: str):
    """HBM bytes per launch of the fused kernel from committed rocprofv3 counter runs,
    or None if none were taken for the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get(dtype)
    if not entry or t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline(boxes, dom, u0, c, nthreads_note: str):
    """The oracle as it stands, one full step (FillBoundary + heat) of the workload."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    m = O.OracleMultiFab(boxes, dom, (1, 1, 1), u0.shape[0], 1)
    m.load_global(u0)
    w = m.copy()
    setup = time.perf_counter() - t0
    # whole steps until about 10 s of host work (at least one step)
    nsteps = 0
    t0 = time.perf_counter()
    while True:
        O.heat_step(m, w, c)
        m, w = w, m
        nsteps += 1
        dt = time.perf_counter() - t0
        if dt >= CPU_SAMPLE_SECONDS or nsteps >= 200:
            break
    cells = sum(int(np.prod(b[3:] - b[:3] + 1)) for b in boxes) * u0.shape[0]
    cores = O.num_threads()
    log(f"cpu baseline: {nsteps} step(s) in {dt:.2f} s (setup {setup:.1f} s), {cores} threads")
    # the same steps on one thread, a shorter sample
    O.set_num_threads(1)
    n1 = 0
    t0 = time.perf_counter()
    try:
        while True:
            O.heat_step(m, w, c)
            m, w = w, m
            n1 += 1
            dt1 = time.perf_counter() - t0
            if dt1 >= CPU_SAMPLE_SECONDS_1T or n1 >= 200:
                break
    finally:
        O.set_num_threads(cores)
    log(f"cpu baseline, one thread: {n1} step(s) in {dt1:.2f} s")
    return {
        "value": round(cells * nsteps / dt / 1e9, 5),
        "unit": "GCell-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{nsteps} full steps (FillBoundary + 7-point update each) of the same workload, FP64, "
                  f"OpenMP over boxes ({nthreads_note})",
        "single_thread": {"value": round(cells * n1 / dt1 / 1e9, 5), "steps": n1},
        "host": {"cpu": host_cpu_model(), "nproc": os.cpu_count()},
    }


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


PROFILE_ARGS = "--steps 20 --warmup 2 --no-cpu-baseline --no-extra --calibrate-copy --zchunk 4 --waves 4 --block 3"


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _short_kernel(name: str) -> str:
    import re
    m = re.search(r"(k_\w+<[^>]*>|k_\w+)", name)
    if m:
        return m.group(1)
    return name.split("(")[0].replace("void ", "")[:60]


def summarize_profiles(d: str) -> int:
    """Summaries of rocprofv3 runs of this script with PROFILE_ARGS: kernel trace
    statistics (DIR/trace), FETCH_SIZE and WRITE_SIZE per dispatch (DIR/fetch,
    DIR/write), and any further counter runs under DIR/pmc_*.  FETCH_SIZE and
    WRITE_SIZE are scaled by what they read for the plain 2 GiB device copy that the
    same runs end with."""
    import glob
    import statistics
    import re

    def one(pattern):
        got = sorted(glob.glob(os.path.join(d, pattern)))
        if not got:
            raise SystemExit(f"missing {pattern} under {d}")
        return got[0]

    logs = {k: open(os.path.join(d, f"{k}.log")).read() for k in ("trace", "fetch", "write")}
    hashes = {k: re.findall(r"kernel source sha256/16: (\w+)", v) for k, v in logs.items()}
    hs = {h for v in hashes.values() for h in v}
    if len(hs) != 1:
        raise SystemExit(f"runs disagree on the kernel source: {hashes}")
    src_hash = hs.pop()
    line = None
    for ln in logs["trace"].splitlines():
        if ln.startswith("{") and '"metric"' in ln:
            line = json.loads(ln)
    if line is None:
        raise SystemExit("no JSON line in the trace run's log")
    dtype = line["dtype"]
    stats = _read_csv(one("trace/*kernel_stats.csv"))
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    heat = [r for r in stats if "k_heat_" in r["Name"] and ", true," in r["Name"]]
    if not heat:
        raise SystemExit("no fused heat kernel in the trace")
    hk = heat[0]["Name"]
    avg_us = float(heat[0]["AverageNs"]) / 1e3

    def per_dispatch(path, counter):
        vals = {}
        for r in _read_csv(path):
            if r["Counter_Name"] == counter:
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    # steady state and first steps apart: a dispatch of the fused kernel that starts
    # more than 20 us after the previous one ended opens a graph launch (the first
    # step of an advance, which reads the x-face neighbours from their rows)
    disp = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                  for r in _read_csv(one("trace/*kernel_trace.csv")) if r["Kernel_Name"] == hk)
    firsts, steady, prev_end = [], [], None
    for st, en in disp:
        (firsts if prev_end is None or st - prev_end > 20000 else steady).append((en - st) / 1e3)
        prev_end = en
    steady_us = statistics.median(steady)
    first_us = statistics.median(firsts)
    ksteps = int(line["steps"])
    graph_us = first_us + (ksteps - 1) * steady_us

    fetch = per_dispatch(one("fetch/*counter_collection.csv"), "FETCH_SIZE")
    write = per_dispatch(one("write/*counter_collection.csv"), "WRITE_SIZE")
    copy_name = next((k for k in fetch if "copyBuffer" in k), None)
    if copy_name is None:
        raise SystemExit("no copy kernel in the counter runs")
    copy_kib = COPY_BYTES / 1024
    big = lambda v: [x for x in v if x > 0.25 * copy_kib / 2]  # the 2 GiB copies, not small ones
    fetch_scale = copy_kib / statistics.median(big(fetch[copy_name]))
    write_scale = copy_kib / statistics.median(big(write[copy_name]))
    f_kib = statistics.median(fetch[hk])
    w_kib = statistics.median(write[hk])
    fetch_b = f_kib * 1024 * fetch_scale
    write_b = w_kib * 1024 * write_scale
    cells = line["config"]["cell_updates_per_step"]
    esize = 8 if dtype == "f64" else 4
    alg = 2 * esize * cells
    args = f"{PROFILE_ARGS} --dtype {dtype}"
    out = os.path.join(ROOT, "profiles", f"heat_fused_512cube_uneven_5comp_{dtype}.md")
    with open(out, "w") as fh:
        fh.write(f"# Fused heat step + FillBoundary, 512^3 random chop, 5 comps, {dtype}\n\n")
        fh.write("Commands (three runs, from the repository root, after `cd /tmp && export TMPDIR=/tmp` for the profiler's files):\n\n")
        for opt in ("--kernel-trace --stats", "--pmc FETCH_SIZE", "--pmc WRITE_SIZE"):
            fh.write(f"    rocprofv3 {opt} --output-format csv -d <out> -o run -- python3 bench.py {args}\n")
        fh.write(f"\nSummarised with `python3 bench.py --summarize-profiles <out>`.  Kernel source sha256/16: `{src_hash}`.\n\n")
        fh.write("## Kernel trace statistics\n\n| kernel | calls | average us | total % |\n|---|---|---|---|\n")
        for r in stats[:10]:
            fh.write(f"| `{_short_kernel(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |\n")
        fh.write("\n## HBM traffic of the fused kernel, per launch (median over dispatches)\n\n")
        fh.write(f"* kernel: `{_short_kernel(hk)}`, average duration {avg_us:.1f} us\n")
        fh.write(f"* copy calibration (`{_short_kernel(copy_name)}`, {COPY_BYTES} bytes read and written): "
                 f"FETCH_SIZE x{fetch_scale:.4f}, WRITE_SIZE x{write_scale:.4f}\n")
        fh.write(f"* FETCH_SIZE {f_kib:.0f} KiB -> {fetch_b / 1e9:.4f} GB read\n")
        fh.write(f"* WRITE_SIZE {w_kib:.0f} KiB -> {write_b / 1e9:.4f} GB written\n")
        fh.write(f"* algorithmic bytes (one read and one write of every cell update): {alg / 1e9:.4f} GB; "
                 f"measured / algorithmic = {(fetch_b + write_b) / alg:.4f}\n")
        fh.write(f"* achieved at the traced average: algorithmic {alg / (avg_us * 1e-6) / 1e9:.0f} GB/s, "
                 f"measured {(fetch_b + write_b) / (avg_us * 1e-6) / 1e9:.0f} GB/s\n")
        fh.write("\n## Steady state and the first step of each advance\n\n")
        fh.write(f"* {len(disp)} dispatches of the fused kernel: {len(firsts)} open a graph launch (the first step of "
                 f"an advance; it reads the x-face neighbours from their rows unless the input's edge mirror is "
                 f"current), {len(steady)} follow one another\n")
        fh.write(f"* median duration: steady state {steady_us:.1f} us ({alg / (steady_us * 1e-6) / 1e9:.0f} GB/s "
                 f"algorithmic, {alg / (steady_us * 1e-6) / 1e9 / (HBM_PEAK_GBS):.4f} of 8 TB/s); first step "
                 f"{first_us:.1f} us\n")
        fh.write(f"* one {ksteps}-step advance from the trace: {graph_us / 1e3:.4f} ms of kernel time = "
                 f"{ksteps * cells / (graph_us * 1e-6) / 1e9:.1f} GCell/s, roofline fraction "
                 f"{ksteps * alg / (graph_us * 1e-6) / 1e9 / HBM_PEAK_GBS:.4f} (the bench line below, timed with "
                 f"events around the graph launch: {line['roofline']['frac']})\n")
        extra_dirs = sorted(x for x in os.listdir(d) if x.startswith("pmc_") and os.path.isdir(os.path.join(d, x)))
        for xd in extra_dirs:
            rows = _read_csv(one(f"{xd}/*counter_collection.csv"))
            per = {}
            for r in rows:
                per.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
            names = sorted({cn for (kn, cn) in per if kn == hk})
            fh.write(f"\n## Counters `{' '.join(names)}` (median per dispatch)\n\n")
            fh.write(f"    rocprofv3 --pmc {' '.join(names)} --output-format csv -d <out>/{xd} -o run -- python3 bench.py {args}\n\n")
            fh.write("| kernel | " + " | ".join(names) + " |\n|---|" + "---|" * len(names) + "\n")
            for kn in (hk, copy_name):
                # the copy kernel: its largest dispatch (the 2 GiB copies, not torch's small ones)
                vals = [(max(per[(kn, cn)]) if kn == copy_name else statistics.median(per[(kn, cn)]))
                        if (kn, cn) in per else float("nan") for cn in names]
                fh.write(f"| `{_short_kernel(kn)}` | " + " | ".join(f"{v:.0f}" for v in vals) + " |\n")
            if "TCC_HIT_sum" in names and "TCC_MISS_sum" in names:
                h = statistics.median(per[(hk, "TCC_HIT_sum")])
                m = statistics.median(per[(hk, "TCC_MISS_sum")])
                fh.write(f"\nL2 hit rate of the fused kernel: {h / (h + m):.4f}\n")
        fh.write(f"\nBench line of the trace run: `{json.dumps({k: line[k] for k in ('value', 'ms_per_step', 'roofline')})}`\n")
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    if t.get("kernel_source_sha256_16") != src_hash:
        t = {"kernel_source_sha256_16": src_hash}
    t[dtype] = {"bytes_per_launch": round(fetch_b + write_b), "fetch_bytes": round(fetch_b),
                "write_bytes": round(write_b), "fetch_scale": round(fetch_scale, 5),
                "write_scale": round(write_scale, 5), "kernel": _short_kernel(hk), "avg_duration_us": round(avg_us, 2),
                "steady_duration_us": round(steady_us, 2), "first_step_duration_us": round(first_us, 2),
                "summary": os.path.relpath(out, ROOT)}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    print(f"wrote {out} and {TRAFFIC_FILE}")
    return 0


EXTRAS_PROFILE_ARGS = "--steps 5 --warmup 1 --no-cpu-baseline --no-serve --calibrate-copy"


def summarize_trace(d: str) -> int:
    """Kernel trace statistics of one rocprofv3 run of this script with EXTRAS_PROFILE_ARGS
    (every extra workload but serving): each kernel's calls and average duration, beside
    the figures the run printed."""
    import glob
    import re
    got = sorted(glob.glob(os.path.join(d, "trace/*kernel_stats.csv")))
    if not got:
        raise SystemExit(f"missing trace/*kernel_stats.csv under {d}")
    stats = _read_csv(got[0])
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    log_text = open(os.path.join(d, "trace.log")).read()
    hashes = set(re.findall(r"kernel source sha256/16: (\w+)", log_text))
    if len(hashes) != 1:
        raise SystemExit(f"no single kernel source hash in the run's log: {hashes}")
    printed = [ln for ln in log_text.splitlines() if ln.startswith("[bench]")]
    out = os.path.join(ROOT, "profiles", "kernels_every_workload.md")
    with open(out, "w") as fh:
        fh.write("# Every kernel of the benchmark's workloads (kernel trace)\n\n")
        fh.write("Command (from the repository root, after `cd /tmp && export TMPDIR=/tmp` for the profiler's files):\n\n")
        fh.write(f"    rocprofv3 --kernel-trace --stats --output-format csv -d <out>/trace -o run -- python3 bench.py {EXTRAS_PROFILE_ARGS}\n\n")
        fh.write(f"Summarised with `python3 bench.py --summarize-trace <out>`.  Kernel source sha256/16: `{hashes.pop()}`.\n")
        fh.write("The workloads: the 512^3 uneven level (fused heat FP64 and FP32, unfused, reductions, the "
                 "variable-coefficient form, the 8th-order step with 4 ghost layers) and the 384^3 level of 64^3 "
                 "boxes (GSRB, multigrid).  Averages mix every launch of a kernel, e.g. all multigrid levels.\n\n")
        fh.write("| kernel | calls | average us | total % |\n|---|---|---|---|\n")
        for r in stats[:40]:
            fh.write(f"| `{_short_kernel(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |\n")
        fh.write("\n## What the run printed\n\n")
        for ln in printed:
            fh.write(f"    {ln}\n")
    print(f"wrote {out}")
    return 0


def per_box_run(bt, I, torch) -> dict:
    """The plain per-box form beside the batched one on the two small workloads:
    CFG0, 64^3 periodic, 8 boxes of 32^3, Gaussian u0, 20 steps; and CFG1, 256^3
    periodic, 64 boxes of 64^3, 3 seeded sine modes, 100 steps.  The per-box form is
    FillBoundary followed by one stencil launch per box each step (the paper's
    fill-then-kernel structure, one grid at a time); the batched form is the fused
    kernel over the flattened tile list, one launch per step, the steps in one graph.
    FP64 and FP32 storage, each timed with events over all its steps."""
    out = {}
    stream = torch.cuda.current_stream()
    for name, n, edge, steps in (("cfg0_64cube_8x32", 64, 32, 20), ("cfg1_256cube_64x64", 256, 64, 100)):
        dom = I.domain_box(n)
        ba = bt.BoxArray.chop(dom, edge)
        if n == 64:
            u0 = I.gaussian(n)[None]
        else:
            u0, _ = I.sine_modes(n, seed=1)
        c = I.heat_c(n)
        cells = n ** 3
        res = {"workload": f"{n}^3 periodic, {len(ba)} boxes of {edge}^3, 1 comp, 1 ghost, {steps} steps"}
        for dname, dt, esize in (("f64", bt.F64, 8), ("f32", bt.F32, 4)):
            g = u0 if dt == bt.F64 else I.round_f32(u0)
            a, b = bt.MultiFab(ba, 1, 1, dt), bt.MultiFab(ba, 1, 1, dt)
            a.from_global(g)

            def per_box(x, y):
                for _ in range(steps):
                    bt.heat_step(x, y, c, fill_first=True)
                    x, y = y, x
                return x

            def timed(fn):
                fn()  # warm-up (captures the graph of the batched form)
                a.from_global(g)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                r = fn()
                e1.record(stream)
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / steps, r

            ms_box, r_box = timed(lambda: per_box(a, b))
            sum_box = r_box.sum(0)
            g_box = r_box.to_global()
            ms_bat, r_bat = timed(lambda: bt.heat_advance(a, b, steps, c))
            same = bool(torch.equal(g_box, r_bat.to_global()))
            gb, gt = cells / (ms_box / 1e3) / 1e9, cells / (ms_bat / 1e3) / 1e9
            res[dname] = {"per_box": {"ms_per_step": round(ms_box, 5), "gcell_s": round(gb, 2),
                                      "hbm_frac": round(gb * 2 * esize / HBM_PEAK_GBS, 4),
                                      "launches_per_step": len(ba) + 1},
                          "batched": {"ms_per_step": round(ms_bat, 5), "gcell_s": round(gt, 2),
                                      "hbm_frac": round(gt * 2 * esize / HBM_PEAK_GBS, 4), "launches_per_step": 1},
                          "batched_over_per_box": round(ms_box / ms_bat, 3),
                          "same_result": same, "sum_after": sum_box}
            log(f"{name} {dname}: per box {ms_box:.4f} ms/step ({gb:.1f} GCell/s), batched {ms_bat:.4f} "
                f"ms/step ({gt:.1f} GCell/s), x{ms_box / ms_bat:.2f}, same result {same}")
            del a, b, r_box, r_bat, g_box
        out[name] = res
    torch.cuda.empty_cache()
    return out


def gsrb_run(bt, I, torch, seed: int, sweeps: int = 20) -> dict:
    """Red-black Gauss-Seidel for -Lap(phi) = f: 384^3 periodic, 216 boxes of 64^3, f a seeded
    zero-mean N(0,1) field rounded to FP32, phi0 = 0, FP32 state, 20 sweeps with a FillBoundary
    before each colour (or its equivalent) and the FP64 residual norm after every sweep.  Forms:
    one_pass (the default: one launch per sweep computes red a plane ahead of black, after the
    ring kernel), two_pass (fused colour passes reading the neighbour boxes directly) and
    fill_then_pass (explicit fills), each with the same result; one_pass also without norms."""
    n = 384
    dom = I.domain_box(n)
    ba = bt.BoxArray.from_boxes(I.regular_chop(dom, 64), dom)
    t0 = time.perf_counter()
    f = I.zero_mean_normal_f32(n, seed=seed)
    log(f"gsrb: source field in {time.perf_counter() - t0:.1f} s")
    h2 = (1.0 / n) ** 2
    out = {"workload": f"{n}^3 periodic, 216 boxes of 64^3, FP32 state, {sweeps} sweeps, FP64 norm each sweep"}
    saved = bt.get_tile_config()
    gsaved = bt.get_gsrb_config()
    forms = (("one_pass", None, gsaved, True), ("one_pass_no_norms", None, gsaved, False),
             ("two_pass", None, (0, gsaved[1], gsaved[2]), True),
             ("fill_then_pass", (saved[0], saved[1], saved[2], 2), (0, gsaved[1], gsaved[2]), True))
    for form, cfg, gcfg, with_norms in forms:
        if cfg:
            bt.set_tile_config(*cfg)
        bt.set_gsrb_config(*gcfg)
        try:
            phi, fm = bt.MultiFab(ba, 1, 1, bt.F32), bt.MultiFab(ba, 1, 1, bt.F32)
            fm.set_val(0.0, with_ghosts=True)
            fm.from_global(f)
            phi.set_val(0.0, with_ghosts=True)
            applies = bt.gsrb_one_pass_applies(phi)
            bt.gsrb_sweeps(phi, fm, h2, 2, with_norms=with_norms)  # warm-up
            phi.set_val(0.0, with_ghosts=True)
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            norms = bt.gsrb_sweeps(phi, fm, h2, sweeps, with_norms=with_norms)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
        finally:
            if cfg:
                bt.set_tile_config(*saved)
            bt.set_gsrb_config(*gsaved)
        cs = n ** 3 * sweeps / (ms / 1e3)
        out[form] = {"ms_per_sweep": round(ms / sweeps, 4), "gcell_sweeps_s": round(cs / 1e9, 2),
                     "hbm_frac_at_12B": round(cs * 12 / (HBM_PEAK_GBS * 1e9), 4), "one_pass": applies}
        if norms:
            out[form].update({"resnorm_first": norms[0], "resnorm_last": norms[-1],
                              "resnorm_h32_first": norms[0] * (1.0 / n) ** 1.5,
                              "resnorm_h32_last": norms[-1] * (1.0 / n) ** 1.5})
        log(f"gsrb {form}: {ms / sweeps:.3f} ms per sweep, {cs / 1e9:.1f} G cell-sweeps/s"
            + (f", norm {norms[0]:.4e} -> {norms[-1]:.4e}" if norms else ""))
        del phi, fm
    del f
    torch.cuda.empty_cache()
    return out


def varcoef_run(bt, I, torch, boxes, dom, u0, ncomp: int, seed: int, steps: int) -> dict:
    """du/dt = div(beta grad u) in the flux form on the same level (FP64, same boxes and
    u0), beta = 0.5 + U(0,1) per cell and component, dt = 0.9 dx^2 / (6 max beta).  The
    kernel's duration per launch is the 2K-step run minus the K-step run over K; its
    algorithmic bytes are u and beta read once and u written once (24 per cell)."""
    n = int(dom[3]) + 1
    ba = bt.BoxArray.from_boxes(boxes, dom)
    a, b, beta = (bt.MultiFab(ba, ncomp, 1, bt.F64) for _ in range(3))
    t0 = time.perf_counter()
    bg = I.uniform(n, ncomp, seed=seed + 1)
    for comp in range(ncomp):
        a.from_global(u0[comp:comp + 1], scomp=comp)
        beta.from_global(bg[comp:comp + 1] + 0.5, scomp=comp)
    del bg
    log(f"varcoef: inputs in {time.perf_counter() - t0:.1f} s")
    dx = 1.0 / n
    dt = 0.9 * dx * dx / (6.0 * 1.5)
    cells = int(sum(int(np.prod(bx[3:] - bx[:3] + 1)) for bx in boxes)) * ncomp
    s0 = a.sum(0)
    bt.heat_varcoef_advance(a, b, beta, 2, dt, dx)  # warm-up, state back in a
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    bt.heat_varcoef_advance(a, b, beta, steps, dt, dx)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ev[2].record(stream)
    res = bt.heat_varcoef_advance(a, b, beta, 2 * steps, dt, dx)
    ev[3].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    per_launch = (ev[2].elapsed_time(ev[3]) - ms) / steps
    drift = abs(res.sum(0) - s0) / abs(s0)
    gbs = 24 * cells / (per_launch / 1e3) / 1e9
    out = {"workload": f"{n}^3 periodic, {len(boxes)} uneven boxes, {ncomp} comps, FP64, beta U(0.5, 1.5)",
           "ms_per_step": round(ms / steps, 5), "kernel_ms_per_launch": round(per_launch, 5),
           "gcell_s": round(cells * steps / (ms / 1e3) / 1e9, 2), "kernel_gbs_at_24B": round(gbs, 1),
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "sum_drift_rel": drift}
    log(f"varcoef: {ms / steps:.3f} ms/step, kernel {per_launch:.3f} ms, {gbs:.0f} GB/s at 24 B/cell, "
        f"drift {drift:.2e}")
    del a, b, beta, ba, res
    torch.cuda.empty_cache()
    return out


def _timed(torch, fn, reps: int) -> float:
    """Milliseconds per call of fn over reps calls (events on the current stream), after one warm-up."""
    fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def mg_levels_breakdown(bt, torch, ba, dt, h2: float, nlevels: int, bottom: int) -> list:
    """Time of each level's part of a V(2,2) cycle, level by level: its 4 GSRB sweeps, the
    restriction (with its FillBoundary) and the prolongation, on a MultiFab of that level's
    boxes; from the fused bottom's first level on, one launch for all the coarser levels
    (a hierarchy built on that level's boxes, whose bottom is its level 0)."""
    rows, cur, h = [], ba, h2
    for lev in range(nlevels):
        cells = int(sum(int(np.prod(b[3:] - b[:3] + 1)) for b in cur.boxes()))
        phi, fm = bt.MultiFab(cur, 1, 1, dt), bt.MultiFab(cur, 1, 1, dt)
        phi.set_val(0.0, with_ghosts=True)
        fm.set_val(1e-3, with_ghosts=True)
        if lev == bottom:
            mgb = bt.Multigrid(cur, dt)
            ms = _timed(torch, lambda: mgb.vcycles(phi, fm, h, 1, with_norms=False), 20)
            rows.append({"levels": f"{lev}-{nlevels - 1}", "cells": cells, "fused_bottom_ms": round(ms, 4)})
            break
        nxt = cur.coarsen(2) if lev + 1 < nlevels else None
        row = {"level": lev, "cells": cells, "boxes": len(cur),
               "sweeps_4_ms": round(_timed(torch, lambda: bt.gsrb_sweeps(phi, fm, h, 4, with_norms=False), 10), 4)}
        if nxt is not None:
            fc = bt.MultiFab(nxt, 1, 1, dt)
            fc.set_val(0.0, with_ghosts=True)
            row["restrict_ms"] = round(_timed(torch, lambda: bt.restrict_residual(phi, fm, h, fc), 10), 4)
            row["prolong_ms"] = round(_timed(torch, lambda: bt.prolong_add(phi, fc), 10), 4)
        rows.append(row)
        if nxt is None:
            break
        cur, h = nxt, 4.0 * h
    return rows


def mg_run(bt, I, torch, seed: int, cycles: int = 5) -> dict:
    """Multigrid V(2,2) cycles for -Lap(phi) = f, 8 bottom sweeps, on GSRB's level (384^3
    periodic, 216 boxes of 64^3: 7 levels down to 216 boxes of one cell) and on 256^3 (64
    boxes of 64^3, 7 levels), f a seeded zero-mean N(0,1) field.  FP64 and FP32 state; time
    per cycle, the residual's mean reduction per cycle, the level where the fused bottom
    starts, and (FP64) each level's part of the cycle."""
    out = {}
    for n in (384, 256):
        dom = I.domain_box(n)
        ba = bt.BoxArray.from_boxes(I.regular_chop(dom, 64), dom)
        f = I.zero_mean_normal_f32(n, seed=seed)
        h2 = (1.0 / n) ** 2
        res = {"workload": f"{n}^3 periodic, {len(ba)} boxes of 64^3, V(2,2), 8 bottom sweeps, {cycles} cycles"}
        for name, dt in (("f64", bt.F64), ("f32", bt.F32)):
            phi, fm = bt.MultiFab(ba, 1, 1, dt), bt.MultiFab(ba, 1, 1, dt)
            fm.set_val(0.0, with_ghosts=True)
            fm.from_global(f)
            mg = bt.Multigrid(ba, dt)
            phi.set_val(0.0, with_ghosts=True)
            r0 = bt.residual_norm(phi, fm, h2)
            mg.vcycles(phi, fm, h2, 1, with_norms=False)  # warm-up
            phi.set_val(0.0, with_ghosts=True)
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mg.vcycles(phi, fm, h2, cycles, with_norms=False)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / cycles
            rn = bt.residual_norm(phi, fm, h2)
            res[name] = {"levels": mg.nlevels, "fused_bottom_from_level": mg.bottom_level,
                         "ms_per_vcycle": round(ms, 4), "resnorm_0": r0,
                         f"resnorm_after_{cycles}": rn, "mean_reduction_per_cycle": (rn / r0) ** (1.0 / cycles)}
            log(f"mg {n}^3 {name}: {mg.nlevels} levels (fused from {mg.bottom_level}), {ms:.3f} ms per V-cycle, "
                f"residual {r0:.3e} -> {rn:.3e}")
            if name == "f64":
                res[name]["per_level"] = mg_levels_breakdown(bt, torch, ba, dt, h2, mg.nlevels, mg.bottom_level)
            del phi, fm, mg
        del f
        out[f"{n}cube"] = res
    torch.cuda.empty_cache()
    return out


def heat8_run(bt, I, torch, boxes, dom, u0, ncomp: int, steps: int = 10) -> dict:
    """The 8th-order heat step (9-cell span, 4 ghost layers) on the same level and u0, FP64,
    c = 0.09, in each form: fused (neighbour boxes read directly, the default where the
    layout allows it), fused with the 4-layer edge mirrors, and fill (FillBoundary of the
    4 layers, then the stencil; the two timed apart)."""
    n = int(dom[3]) + 1
    ba = bt.BoxArray.from_boxes(boxes, dom)
    a, b = bt.MultiFab(ba, ncomp, 4, bt.F64), bt.MultiFab(ba, ncomp, 4, bt.F64)
    for comp in range(ncomp):
        a.from_global(u0[comp:comp + 1], scomp=comp)
    cells = int(sum(int(np.prod(bx[3:] - bx[:3] + 1)) for bx in boxes)) * ncomp
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def per_step(fn):
        fn(2)
        torch.cuda.synchronize()
        ev[0].record(stream)
        fn(steps)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    fill_form = per_step(lambda k: bt.heat8_advance(a, b, k, 0.09, form="fill"))
    fill = per_step(lambda k: [a.fill_boundary() for _ in range(k)])
    fused_ok = bt.heat8_fused_ok(a)
    fused = per_step(lambda k: bt.heat8_advance(a, b, k, 0.09, form="fused")) if fused_ok else None
    try:
        mirror = per_step(lambda k: bt.heat8_advance(a, b, k, 0.09, form="fused_mirror"))
    except bt.BoxtileError:  # a box narrower than 8 cells in x
        mirror = None
    form = bt.heat8_auto_form(a)
    ms = fused if form == "fused" else fill_form
    kern = fill_form - fill
    gbs = 16 * cells / (ms / 1e3) / 1e9
    out = {"workload": f"{n}^3 periodic, {len(boxes)} uneven boxes, {ncomp} comps, 4 ghost layers, FP64",
           "form": form, "ms_per_step": round(ms, 4),
           "fused_form_ms_per_step": round(fused, 4) if fused_ok else None,
           "fused_mirror_form_ms_per_step": round(mirror, 4) if mirror is not None else None,
           "gcell_s": round(cells / (ms / 1e3) / 1e9, 2), "step_gbs_at_16B": round(gbs, 1),
           "step_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "fill_form": {"ms_per_step": round(fill_form, 4), "fill_ms": round(fill, 4), "stencil_ms": round(kern, 4),
                         "stencil_gbs_at_16B": round(16 * cells / (kern / 1e3) / 1e9, 1)}}
    log(f"heat8: {ms:.3f} ms/step (default: {form} form, {gbs:.0f} GB/s at 16 B/cell); fill form {fill_form:.3f} ms "
        f"(fill {fill:.3f}, stencil {kern:.3f}); fused form " + (f"{fused:.3f} ms" if fused_ok else "n/a") +
        "; with the 4-layer mirrors " + (f"{mirror:.3f} ms" if mirror is not None else "n/a"))
    del a, b, ba
    torch.cuda.empty_cache()
    return out


def paper_shape_run(bt, I, torch, steps: int = 1000) -> dict:
    """The paper's own workload as context: one 128^3 periodic box, FP64, 1000 fused
    FillBoundary + heat steps (the paper times the kernel alone, on CPUs), with the tile
    shape the autotuner picks for it."""
    n = 128
    dom = I.domain_box(n)
    ba = bt.BoxArray.chop(dom, n)
    a, b = bt.MultiFab(ba, 1, 1, bt.F64), bt.MultiFab(ba, 1, 1, bt.F64)
    c = I.heat_c(n)
    best, _ = bt.autotune(ba, a, b, c)  # its own tile shape, as for the main workload (overwrites a, b)
    a.from_global(I.gaussian(n))
    bt.heat_advance(a, b, steps, c)  # captures the graph; 1000 even: the state is back in a
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    bt.heat_advance(a, b, steps, c)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    g = n ** 3 * steps / (ms / 1e3) / 1e9
    out = {"workload": f"{n}^3 periodic, one box, FP64, {steps} fused steps", "ms": round(ms, 3),
           "gcell_s": round(g, 2), "tile_shape": list(best),
           "paper_cpu_context": {"one_core_tiled_gcell_s": 0.247, "twelve_threads_tiled_gcell_s": 2.2,
                                 "note": "kernel time only, Ivy Bridge (Table 1 and the 12-thread speedup)"}}
    log(f"paper's shape: 128^3 x {steps} steps in {ms:.1f} ms, {g:.1f} GCell/s (tile shape {tuple(best)})")
    del a, b, ba
    torch.cuda.empty_cache()
    return out


def copy_line(bt, torch, nbytes: int = COPY_BYTES) -> dict:
    """Device copies of nbytes timed with events, the attainable HBM line: the library's
    plain streaming copy (16-byte lanes, 4 KB per workgroup) and torch's copy_."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    out = {"bytes": nbytes}
    for name, fn in (("library", lambda: bt.device_copy(dst, src)), ("torch", lambda: dst.copy_(src))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        gbs = 2 * nbytes / (ms / 1e3) / 1e9
        out[name] = {"ms": round(ms, 4), "gbs_read_plus_write": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"device copy ({name}): {gbs:.0f} GB/s read + write")
    assert torch.equal(dst, src)
    del src, dst
    torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--n", type=int, default=512, help="domain edge")
    ap.add_argument("--ncomp", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=None)
    ap.add_argument("--waves", type=int, default=None)
    ap.add_argument("--persist", type=int, default=None)
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--zsteps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32 and unfused measurements")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving runs")
    ap.add_argument("--no-gsrb", action="store_true", help="skip the GSRB smoother run")
    ap.add_argument("--no-varcoef", action="store_true", help="skip the variable-coefficient flux-form run")
    ap.add_argument("--no-mg", action="store_true", help="skip the multigrid V-cycle run")
    ap.add_argument("--no-heat8", action="store_true", help="skip the 8th-order stencil run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with three plain device copies of 2 GiB (reference for HBM byte counters)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="no GPU: turn a kernel-trace run of this script with EXTRAS_PROFILE_ARGS (DIR/trace, "
                         "DIR/trace.log) into profiles/kernels_every_workload.md")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="no GPU: turn rocprofv3 output of this script (DIR/trace, DIR/fetch, DIR/write) into "
                         "the summary and traffic files under profiles/")
    args = ap.parse_args()

    if args.summarize_profiles:
        return summarize_profiles(args.summarize_profiles)
    if args.summarize_trace:
        return summarize_trace(args.summarize_trace)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import torch
    from paper_1604_03570_amd import boxtile as bt
    from paper_1604_03570_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    explicit = bool(args.zchunk or args.waves or args.persist is not None or args.block is not None or args.zsteps)
    if explicit:
        z, w, p, b, zs = bt.get_tile_config()
        bt.set_tile_config(args.zchunk or z, args.waves or w, p if args.persist is None else args.persist,
                           b if args.block is None else args.block, args.zsteps or zs)
    cfg_tile = bt.get_tile_config()
    log(f"kernel source sha256/16: {kernel_source_hash()}")

    n, ncomp = args.n, args.ncomp
    dom = I.domain_box(n)
    boxes = I.random_chop(dom, 16, 128, 8, seed=args.seed)
    c = I.heat_c(n)
    log(f"workload: {n}^3, {len(boxes)} boxes, {ncomp} comps, dtype {args.dtype}, "
        f"tile shape {'fixed ' + str(cfg_tile) if explicit else 'autotuned'}")
    t0 = time.perf_counter()
    u0 = I.uniform(n, ncomp, seed=args.seed)
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s")
    cells = int(sum(int(np.prod(b[3:] - b[:3] + 1)) for b in boxes)) * ncomp

    def run(dtype_name: str, steps: int, warmup: int):
        dt = bt.F64 if dtype_name == "f64" else bt.F32
        ba = bt.BoxArray.from_boxes(boxes, dom)
        a, b = bt.MultiFab(ba, ncomp, 1, dt), bt.MultiFab(ba, ncomp, 1, dt)
        tuned = None
        if not explicit:  # pick the tile shape on this workload before loading the data
            t0 = time.perf_counter()
            a.set_val(0.5)
            b.set_val(0.5)
            best, table = bt.autotune(ba, a, b, c, trial_steps=3)
            tuned = {"best": list(best), "seconds": round(time.perf_counter() - t0, 2),
                     "table": [[list(k), round(v, 4)] for k, v in table]}
            log(f"{dtype_name}: autotuned tile shape {best} in {tuned['seconds']} s")
        for comp in range(ncomp):  # one component at a time keeps the staging copy small
            a.from_global(u0[comp:comp + 1], scomp=comp)
        torch.cuda.synchronize()
        if warmup:
            x = bt.heat_advance(a, b, warmup, c)
        else:
            x = a
        y = b if x is a else a
        torch.cuda.synchronize()
        s0 = x.sum(0)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # capture the K-step graph outside the timed region; with K odd run it twice
        # so that the state is back in x and the timed call reuses the same graph
        for _ in range(1 if steps % 2 == 0 else 2):
            bt.heat_advance(x, y, steps, c)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(stream)
        res = bt.heat_advance(x, y, steps, c)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = e0.elapsed_time(e1)
        drift = abs(res.sum(0) - s0) / abs(s0)
        # marginal duration of one step: a 2K-step graph minus the K-step one (both
        # measured with events on this stream); the first step of an advance (it
        # reads the x-face neighbours from their rows, no edge mirror of the
        # starting state exists yet) and the graph launch drop out of it
        cur = res
        oth = a if cur is b else b
        bt.heat_advance(cur, oth, 2 * steps, c)  # captures the 2K-step graph; 2K even: state back in cur
        torch.cuda.synchronize()
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        bt.heat_advance(cur, oth, 2 * steps, c)
        e3.record(stream)
        torch.cuda.synchronize()
        per_launch_ms = (e2.elapsed_time(e3) - ms) / steps
        # five more timings of the K-step graph from cur (the same work each time):
        # their median and minimum
        reps = []
        for _ in range(5):
            e2.record(stream)
            bt.heat_advance(cur, oth, steps, c)
            e3.record(stream)
            torch.cuda.synchronize()
            reps.append(e2.elapsed_time(e3) / steps)
        return ms, wall, drift, ba, a, b, per_launch_ms, tuned, reps

    ms, wall, drift, ba, a, b, per_launch_ms, tuned, reps = run(args.dtype, args.steps, args.warmup)
    esize = 8 if args.dtype == "f64" else 4
    sec = ms / 1e3
    value = cells * args.steps / sec / 1e9
    alg_bytes = 2 * esize * cells  # read u once, write u_new once
    # algorithmic bytes per launch over the average launch time of the timed region
    # (one launch per step): the same figure as value x b_alg
    achieved = alg_bytes / (sec / args.steps) / 1e9
    marginal_gbs = alg_bytes / (per_launch_ms / 1e3) / 1e9
    traffic = measured_traffic(args.dtype)
    log(f"{args.dtype}: {ms:.3f} ms for {args.steps} steps (wall {wall * 1e3:.3f} ms), "
        f"{value:.1f} GCell/s, {achieved:.0f} GB/s, sum drift {drift:.2e}")

    extra = {"sum_drift_rel": drift, "wall_ms_timed": round(wall * 1e3, 4),
             "tile_shape": tuned["best"] if tuned else list(cfg_tile), "autotune": tuned,
             "nboxes": len(boxes),
             "marginal_per_launch": {"ms": round(per_launch_ms, 5), "gbs": round(marginal_gbs, 1),
                                     "frac": round(marginal_gbs / HBM_PEAK_GBS, 4),
                                     "note": "(T(2K-step graph) - T(K-step graph)) / K: one step of a long run, "
                                             "without the first step of an advance and the graph launch"},
             "ms_per_step_repeats": {"n": len(reps), "median": round(float(np.median(reps)), 5),
                                     "min": round(min(reps), 5)}}
    if not args.no_extra:
        # unfused form: fill kernel and stencil kernel timed apart (fill fraction)
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        reps = 10
        for _ in range(2):
            bt.heat_step_unfused(a, b, c)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            a.fill_boundary()
        ev[1].record(stream)
        for _ in range(reps):
            bt.heat_step_unfused(a, b, c)
        ev[2].record(stream)
        torch.cuda.synchronize()
        fill_ms = ev[0].elapsed_time(ev[1]) / reps
        unfused_ms = ev[1].elapsed_time(ev[2]) / reps
        extra["unfused_ms_per_step"] = round(unfused_ms, 4)
        extra["unfused_fill_ms"] = round(fill_ms, 4)
        extra["unfused_fill_fraction"] = round(fill_ms / unfused_ms, 4)
        extra["unfused_gcell_s"] = round(cells / (unfused_ms / 1e3) / 1e9, 2)
        # reductions over one component (valid cells; FP64 accumulation)
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        a.reduce_async(0, "sum", out)
        torch.cuda.synchronize()
        ev[2].record(stream)
        for _ in range(reps):
            a.reduce_async(0, "sum", out)
        ev[3].record(stream)
        torch.cuda.synchronize()
        red_ms = ev[2].elapsed_time(ev[3]) / reps
        comp_bytes = cells // ncomp * esize
        extra["reduce_sum_ms"] = round(red_ms, 4)
        extra["reduce_sum_gbs"] = round(comp_bytes / (red_ms / 1e3) / 1e9, 1)
        log(f"reduce sum (one component): {red_ms:.3f} ms, {comp_bytes / (red_ms / 1e3) / 1e9:.0f} GB/s")
        log(f"unfused: {unfused_ms:.3f} ms/step, fill {fill_ms:.3f} ms ({fill_ms / unfused_ms:.1%})")
        del a, b, ba
        torch.cuda.empty_cache()
        if args.dtype == "f64":
            ms32, _, drift32, ba32, a32, b32, _, tuned32, _ = run("f32", args.steps, args.warmup)
            v32 = cells * args.steps / (ms32 / 1e3) / 1e9
            extra["f32_gcell_s"] = round(v32, 2)
            extra["f32_ms_per_step"] = round(ms32 / args.steps, 5)
            extra["f32_hbm_frac"] = round(v32 * 8 / HBM_PEAK_GBS, 4)
            extra["f32_sum_drift_rel"] = drift32
            extra["f32_tile_shape"] = tuned32["best"] if tuned32 else list(cfg_tile)
            log(f"f32: {v32:.1f} GCell/s")
            del a32, b32, ba32
            torch.cuda.empty_cache()

    if not args.no_extra and args.dtype == "f64":
        extra["copy_line"] = copy_line(bt, torch)
        extra["paper_shape"] = paper_shape_run(bt, I, torch)
        extra["per_box_baseline"] = per_box_run(bt, I, torch)

    if not args.no_extra and not args.no_varcoef and args.dtype == "f64":
        extra["varcoef"] = varcoef_run(bt, I, torch, boxes, dom, u0, ncomp, args.seed, 20)
    if not args.no_extra and not args.no_heat8 and args.dtype == "f64":
        extra["heat8"] = heat8_run(bt, I, torch, boxes, dom, u0, ncomp)

    if not args.no_extra and not args.no_gsrb:
        extra["gsrb"] = gsrb_run(bt, I, torch, args.seed)

    if not args.no_extra and not args.no_mg:
        extra["mg"] = mg_run(bt, I, torch, args.seed)

    if not args.no_extra and not args.no_serve:
        # serving: 2000 independent periodic heat problems, Poisson arrivals at 200/s,
        # edge 32..256, box edge 32 or 64, 10..200 steps, FP32/FP64; continuous batching
        # with HBM admission at a generous and a tight budget
        from paper_1604_03570_amd import serve as S
        reqs = I.request_stream(2000, 200.0, seed=args.seed)
        sv = {"requests": len(reqs), "rate_per_s": 200.0, "offered_gcell_s": round(S.offered_load(reqs) / 1e9, 3)}
        for name, budget, steps in (("budget_64GiB", 64 << 30, 16), ("budget_1GiB", 1 << 30, 16),
                                    ("budget_64GiB_one_step_per_launch", 64 << 30, 1)):
            sv[name] = S.Server(budget, max_slots=64, max_steps=steps).run(reqs).summary()
            log(f"serve {name}: p50 {sv[name]['p50_ms']} ms, p99 {sv[name]['p99_ms']} ms, "
                f"{sv[name]['throughput_gcell_s']} GCell/s")
        extra["serve"] = sv
        extra["serve_p50_ms"] = sv["budget_64GiB"]["p50_ms"]
        extra["serve_p99_ms"] = sv["budget_64GiB"]["p99_ms"]

    if args.calibrate_copy:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # give the scale of those counters on this device
        torch.cuda.empty_cache()
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {COPY_BYTES} bytes")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(boxes, dom, u0, c, f"OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS', 'unset')}")

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GCell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"batched heat step + FillBoundary (fused, one launch per step, HIP graph): {n}^3 periodic "
                        f"domain, seeded recursive chop into {len(boxes)} boxes of edge 16-128, {ncomp} comps, "
                        f"1 ghost, U(0,1) initial data, {args.dtype}",
            "domain": n, "nboxes": len(boxes), "ncomp": ncomp, "nghost": 1, "seed": args.seed,
            "cell_updates_per_step": cells,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
