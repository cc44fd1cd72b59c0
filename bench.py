"""Throughput benchmark of the two-component Shan-Chen step on one MI355X.

Workload: D3Q19 droplet on a 128^3 periodic box, R0 = 24, tau = 1,
g_AB = G c_s^2 = 1.8 (symmetric, psi = n), E6 force stencil, populations
stored and updated in FP32 (structure-of-arrays), synthetic tanh initial
profile of Sec. 4 between the bulk concentrations of a converged flat
interface (the paper's two-stage initialisation, first stage run on the GPU
before timing).  A timed step is one lattice update of both components
(stream + concentrations + Shan-Chen force + common velocity + BGK/Guo
collide); the FP64 statistics, the pressure-tensor / sigma[R] / R_s
reductions and the convergence criteria (Delta P change, du, droplet centre)
run at the paper's monitoring cadence: whenever the run's step count reaches a
multiple of 2^11 (Sec. 4), inside the timed region when that falls there, and
once after it for the reported observables otherwise.

Prints one JSON line: MLUPS (million lattice-site updates per second, both
components), the roofline of the step kernel (algorithmic bytes 4 Q s per
site = 304 B for FP32 over the event-timed kernel time, against the 8 TB/s
HBM peak), the HBM traffic measured by rocprofv3 counters for the same
kernel source when available, and the FP64 CPU oracle timed on a bounded
sample of the same workload.  Beside it go the step rates of the other
storage formats (FP64, FP16 and BF16 offsets) on the same droplet and of the
48-member batched sweep (the moment two-pass over member chunks, in 64-step
graphs), each over a short timed run.
"""
import argparse
import csv
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS = {"auto": 0, "two_pass": 1, "fused": 2, "fused_repull": 3, "fused_pipe": 4,
           "fused_mom": 5, "fused_mom_pipe": 6, "two_pass_mom": 7}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}
OBS_EVERY = 2048
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "step_e6_f32_128cube_traffic.txt")
TRACE_MD = os.path.join(ROOT, "profiles", "step_e6_f32_128cube_kernel_trace.md")
# the profiled workloads: the 128^3 droplet in each storage (the benchmark's
# FP32 one without a suffix) and the 48-member batched sweep
# each pins its design, so that the trace and the counter runs profile the
# same kernels (the autotuner's pick between the direct and the LDS-staged
# pass 2 can differ from run to run): the LDS-staged pass 2 for the 16-bit
# formats (the pick of their bench variants), the direct one for FP32
PROFILE_RUNS = {"f32": "--storage f32 --kernel two_pass_mom",
                "f16_offset": "--storage f16_offset --kernel two_pass_mom --tile 64 8 8",
                "bf16_offset": "--storage bf16_offset --kernel two_pass_mom --tile 64 8 8",
                "f16_node": "--storage f16_node --kernel two_pass_mom --tile 64 8 8",
                "bf16_node": "--storage bf16_node --kernel two_pass_mom --tile 64 8 8",
                "batch48": "--batch-only"}


def profile_commands(tag):
    """The rocprofv3 commands whose output summarize_profiles reads for one
    profiled workload (repository root, one MI355X)."""
    sub = "" if tag == "f32" else "_" + tag
    run = PROFILE_RUNS[tag]
    return {
        "trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof{sub}_trace "
                 f"-o trace -- python3 bench.py --steps 300 --warmup 20 --cpu-steps 0 --variant-steps 0 --init tanh {run}",
        "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof{sub}_fetch -o fetch "
                 f"-- python3 bench.py --steps 20 --warmup 5 --cpu-steps 0 --variant-steps 0 --init tanh {run}",
        "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof{sub}_write -o write "
                 f"-- python3 bench.py --steps 20 --warmup 5 --cpu-steps 0 --variant-steps 0 --init tanh {run}",
        "copy_fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof_copy_fetch "
                      "-o cfetch -- python3 bench.py --copy-calib 1024",
        "copy_write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof_copy_write "
                      "-o cwrite -- python3 bench.py --copy-calib 1024",
    }


PROFILE_COMMANDS = profile_commands("f32")
KERNEL_SOURCES = ["paper_2112_02574_amd/csrc/step_kernels.hip",
                  "paper_2112_02574_amd/csrc/fused_impl.h",
                  "paper_2112_02574_amd/csrc/fused_inst.hip",
                  "paper_2112_02574_amd/csrc/fused_kernels.hip",
                  "paper_2112_02574_amd/csrc/site_ops.h",
                  "paper_2112_02574_amd/csrc/lattice.h"]
G_SYM = ((0.0, 1.8), (1.8, 0.0))
G_ASYM = ((-0.2, 1.8), (1.8, 0.0))


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n_sites):
    """HBM bytes per step launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("sites") != n_sites:
        return None
    return t.get("hbm_bytes_per_launch")


def _finite(v):
    return v if isinstance(v, (int, float)) and v == v and abs(v) != float("inf") else None


STEP_KERNEL = re.compile(r"scmc::kb?_(fused|density|collide|moments|collide_mom)(_buf|_lds)?<")


def summarize_profiles(outdir, tag="f32", L=128):
    """Write the profiles/ summaries from the rocprofv3 CSV output of the
    commands of profile_commands(tag) (run from the repository root).  A step
    is one launch of each step kernel (one for the fused designs, two for the
    two-pass ones, two per member chunk for the batch); durations and
    counters are summed over them."""
    import csv
    from paper_2112_02574_amd import inputs
    sub = "" if tag == "f32" else "_" + tag
    cmds = profile_commands(tag)
    if tag == "batch48":
        N = sum(m["L"] ** 3 for m in inputs.batch_members())
        bps, title = 304, "48-member batched sweep (48^3..160^3 droplets), FP32 populations"
    else:
        N = L ** 3
        bps = STORAGE_BYTES[tag]
        title = f"D3Q19 E6 droplet {L}^3, {tag} populations"
    traffic_json = TRAFFIC_JSON if tag == "f32" else os.path.join(
        ROOT, "profiles", f"step_e6_{tag}_traffic.txt")
    trace_md = TRACE_MD if tag == "f32" else os.path.join(
        ROOT, "profiles", f"step_e6_{tag}_kernel_trace.md")

    def rows(sub, suffix):
        d = os.path.join(outdir, sub)
        name = [f for f in os.listdir(d) if f.endswith(suffix)][0]
        return list(csv.DictReader(open(os.path.join(d, name))))

    def mean_counter(sub, prefix):
        v = [float(r["Counter_Value"]) for r in rows(sub, "_counter_collection.csv")
             if r["Kernel_Name"].startswith(prefix)]
        return sum(v) / len(v), len(v)

    stats = rows(f"prof{sub}_trace", "_kernel_stats.csv")
    step_rows = [r for r in stats if STEP_KERNEL.search(r["Name"])
                 and "density64" not in r["Name"] and "kb_" not in r["Name"]]
    names = [r["Name"].split("(")[0] for r in step_rows]
    step_us = sum(float(r["AverageNs"]) for r in step_rows) / 1e3
    per_step = 1
    if tag == "batch48":
        # the batch's two-pass launches (its process also runs the FP64 flat
        # stages and the autotuner's candidates): one pass 1 and one pass 2
        # per member chunk and step (tile-list kernels kb_*, or for a chunk
        # of one member the single-lattice ones), several steps chunk by
        # chunk.  The trace run's last 300 steps are the launches from the
        # end back to where the pass-1 launches have covered every member's
        # sites (in 256-site blocks) 300 times; the step time is their
        # summed duration over 300
        seq = [r for r in rows(f"prof{sub}_trace", "_kernel_trace.csv")
               if re.search(r"scmc::kb?_(moments|collide_mom)_buf<", r["Kernel_Name"])]
        seq.sort(key=lambda r: int(r["Start_Timestamp"]))
        need = 300 * sum(-(-m["L"] ** 3 // 256) * 256 for m in inputs.batch_members())
        got, i = 0, len(seq)
        while got < need and i > 0:
            i -= 1
            if "moments" in seq[i]["Kernel_Name"]:
                got += (int(seq[i]["Grid_Size_X"]) * int(seq[i]["Grid_Size_Y"])
                        * int(seq[i]["Grid_Size_Z"]))
        if got != need:
            raise SystemExit(f"batch trace: pass-1 launches cover {got} sites, not {need}")
        window = seq[i:]
        per_step = round(len(window) / 300)
        names = sorted({r["Kernel_Name"].split("(")[0] for r in window})
        step_us = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                      for r in window) / 300 / 1e3
    fetch = write = 0.0
    nf = nw = 0
    have_counters = os.path.isdir(os.path.join(outdir, f"prof{sub}_fetch")) and any(
        f.endswith("_counter_collection.csv")
        for f in os.listdir(os.path.join(outdir, f"prof{sub}_fetch")))
    for nm in (names if have_counters else []):
        f, a = mean_counter(f"prof{sub}_fetch", nm)
        w, b = mean_counter(f"prof{sub}_write", nm)
        # a batch step launches each kernel once per member chunk (the counter
        # runs of the batch take 20 warm-up and 20 timed steps)
        per = max(1, round(a / 40)) if tag == "batch48" else 1
        fetch, write, nf, nw = fetch + f * per, write + w * per, nf + a, nw + b
    cf, _ = mean_counter("prof_copy_fetch", "__amd_rocclr_copyBuffer")
    cw, _ = mean_counter("prof_copy_write", "__amd_rocclr_copyBuffer")
    copy_bytes = 1024 * (1 << 20)
    sf, sw = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    hbm = fetch * 1024 * sf + write * 1024 * sw
    if not have_counters:
        lines = ["# Kernel trace: " + title, "",
                 "Command (repository root, one MI355X):", "", "    " + cmds["trace"], "",
                 "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
        for r in stats[:8]:
            lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %.2f |" % (
                r["Name"].split("(")[0], r["Calls"], float(r["AverageNs"]) / 1e3,
                float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
        lines += ["", "Step kernels: %s." % ", ".join("`%s`" % n for n in names), "",
                  "One step (the %d launches of a step, summed, averaged over the trace run's last "
                  "300 steps): %.1f us = %.0f MLUPS; algorithmic %d B/site -> %.0f GB/s (%.1f%% of "
                  "8 TB/s)." % (per_step, step_us, N / step_us, bps, bps * N / step_us / 1e3,
                                bps * N / step_us / 1e3 / 80),
                  "", "No HBM traffic counters: rocprofv3 --pmc runs of this program ended with a "
                  "segmentation fault of the profiled process before the first step.", ""]
        with open(trace_md, "w") as fh:
            fh.write("\n".join(lines))
        print(open(trace_md).read())
        return
    traffic = {"kernels": names, "sites": N, "dispatches": {"fetch": nf, "write": nw},
               "fetch_size_kib_per_step": round(fetch, 1),
               "write_size_kib_per_step": round(write, 1),
               "copy_calibration": {"bytes": copy_bytes, "fetch_size_kib": round(cf, 1),
                                    "write_size_kib": round(cw, 1), "fetch_scale": round(sf, 4),
                                    "write_scale": round(sw, 4)},
               "hbm_bytes_per_launch": round(hbm), "algorithmic_bytes_per_launch": bps * N,
               "ratio_to_algorithmic": round(hbm / (bps * N), 4),
               "kernel_source_hash": kernel_source_hash(),
               "commands": [cmds[k] for k in ("fetch", "write", "copy_fetch", "copy_write")]}
    with open(traffic_json, "w") as fh:
        json.dump(traffic, fh, indent=1)
        fh.write("\n")
    lines = ["# Kernel trace: " + title, "",
             "Command (repository root, one MI355X):", "", "    " + cmds["trace"], "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in stats[:8]:
        lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %.2f |" % (
            r["Name"].split("(")[0], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    lines += ["", "Step kernels: %s." % ", ".join("`%s`" % n for n in names),
              "", "One step: %.1f us = %.0f MLUPS; algorithmic %d B/site -> %.0f GB/s "
              "(%.1f%% of 8 TB/s)." % (step_us, N / step_us, bps, bps * N / step_us / 1e3,
                                       bps * N / step_us / 1e3 / 80),
              "", "HBM traffic per step (rocprofv3 counters summed over the step kernels, scaled by a "
              "1 GiB copy): FETCH_SIZE %.0f KiB x %.3f + WRITE_SIZE %.0f KiB x %.3f = %.1f MB, "
              "%.3f x the algorithmic %.1f MB." % (
                  fetch, sf, write, sw, hbm / 1e6, hbm / (bps * N), bps * N / 1e6), ""]
    if tag == "batch48":
        lines[-1:-1] = ["A batch step launches pass 1 and pass 2 once per member chunk (%d launches: a "
                        "chunk of one member as a single lattice, the others one workgroup per 256-site "
                        "tile); the step time is the launches' summed duration "
                        "over the trace run's last 300 steps, divided by 300, and the trace's averages "
                        "above are per chunk." % per_step, ""]
    with open(trace_md, "w") as fh:
        fh.write("\n".join(lines))
    print(open(trace_md).read())


# the FP32 designs compared at 128^3: kernel trace, FETCH/WRITE traffic and
# the SQ instruction mix of each (profiles/step_e6_f32_128cube_designs.md)
DESIGN_RUNS = {"two_pass_mom": "--storage f32 --kernel two_pass_mom",
               "two_pass_mom_lds": "--storage f32 --kernel two_pass_mom --tile 64 8 8",
               "fused_mom": "--storage f32 --kernel fused_mom --tile 128 4 16",
               "two_pass": "--storage f32 --kernel two_pass"}
SQ_COUNTERS = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR "
               "SQ_INSTS_SALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES")


def design_profile_commands(name):
    run = DESIGN_RUNS[name]
    base = "python3 bench.py --steps 20 --warmup 5 --cpu-steps 0 --variant-steps 0 --init tanh " + run
    return {
        "trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/dprof_{name}_trace "
                 f"-o trace -- python3 bench.py --steps 300 --warmup 20 --cpu-steps 0 --variant-steps 0 "
                 f"--init tanh {run}",
        "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/dprof_{name}_fetch -o fetch -- {base}",
        "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/dprof_{name}_write -o write -- {base}",
        "sq": f"rocprofv3 --pmc {SQ_COUNTERS} --output-format csv -d gpurun_out/dprof_{name}_sq -o sq -- {base}",
    }


def summarize_designs(outdir, L=128):
    """profiles/step_e6_f32_128cube_designs.md from the design_profile_commands
    outputs (and the copy calibration of the FP32 profile)."""
    N = L ** 3

    def rows(sub, suffix):
        d = os.path.join(outdir, sub)
        name = [f for f in os.listdir(d) if f.endswith(suffix)][0]
        return list(csv.DictReader(open(os.path.join(d, name))))

    def mean_by_kernel(sub):
        acc = {}
        for r in rows(sub, "_counter_collection.csv"):
            k = r["Kernel_Name"].split("(")[0]
            acc.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}

    cf = mean_by_kernel("prof_copy_fetch")["__amd_rocclr_copyBuffer"]["FETCH_SIZE"]
    cw = mean_by_kernel("prof_copy_write")["__amd_rocclr_copyBuffer"]["WRITE_SIZE"]
    sf, sw = (1 << 30) / (cf * 1024), (1 << 30) / (cw * 1024)
    lines = ["# FP32 step designs on the 128^3 droplet: time, traffic, instruction mix", "",
             "D3Q19 E6 droplet 128^3, FP32 populations, tau = 1. Per step kernel: the mean duration "
             "of the trace run, its LDS per workgroup, HBM traffic from FETCH_SIZE / WRITE_SIZE "
             "scaled by a 1 GiB copy (FETCH x%.3f, WRITE x%.3f), and the instructions the SQ counters "
             "count per 64 sites (one wavefront's worth; the designs give a wavefront different "
             "numbers of sites)." % (sf, sw), "",
             "| design | kernel | us | LDS B/WG | HBM MB | VALU | LDS | VMEM rd | VMEM wr | SALU |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    summary = []
    copy_line = None
    for name in DESIGN_RUNS:
        cmds = design_profile_commands(name)
        trace = rows(f"dprof_{name}_trace", "_kernel_trace.csv")
        stats = rows(f"dprof_{name}_trace", "_kernel_stats.csv")
        fetch, write, sq = (mean_by_kernel(f"dprof_{name}_{k}") for k in ("fetch", "write", "sq"))
        step_us = hbm = 0.0
        for st in stats:
            k = st["Name"].split("(")[0]
            if "k_pull_copy<3, float>" in k and copy_line is None:
                us = float(st["AverageNs"]) / 1e3
                copy_line = (us, 304 * N / (us * 1e-6) / 1e9)
            if not STEP_KERNEL.search(k) or "density64" in k or "kb_" in k:
                continue
            t = next(r for r in trace if r["Kernel_Name"].split("(")[0] == k)
            lds = int(t["LDS_Block_Size"])
            us = float(st["AverageNs"]) / 1e3
            h = (fetch.get(k, {}).get("FETCH_SIZE", 0) * sf + write.get(k, {}).get("WRITE_SIZE", 0) * sw) * 1024
            q = sq.get(k, {})
            per = N / 64.0
            step_us += us
            hbm += h
            lines.append("| %s | `%s` | %.1f | %d | %.0f | %.0f | %.0f | %.1f | %.1f | %.0f |" % (
                name, k.replace("void scmc::", ""), us, lds, h / 1e6,
                q.get("SQ_INSTS_VALU", 0) / per, q.get("SQ_INSTS_LDS", 0) / per,
                q.get("SQ_INSTS_VMEM_RD", 0) / per, q.get("SQ_INSTS_VMEM_WR", 0) / per,
                q.get("SQ_INSTS_SALU", 0) / per))
        summary.append((name, step_us, hbm, cmds))
    lines += ["", "| design | us per step | MLUPS | % of 8 TB/s at 304 B/site | HBM bytes / algorithmic |",
              "|---|---|---|---|---|"]
    for name, us, hbm, _ in summary:
        lines.append("| %s | %.1f | %.0f | %.1f | %.3f |" % (
            name, us, N / us, 304 * N / (us * 1e-6) / 8e12 * 100, hbm / (304 * N)))
    if copy_line:
        lines += ["", "Copy ceiling: `scmc_pull_copy` (the populations of one buffer copied to the other "
                  "with the pull shifts, one site per lane, the step's access pattern without its "
                  "arithmetic) takes %.1f us on the same buffers: %.0f GB/s, %.1f%% of 8 TB/s. "
                  "It runs after the timed steps of the first design's trace run." % (
                      copy_line[0], copy_line[1], copy_line[1] / 80)]
    lines += ["", "Commands (repository root, one MI355X), per design:", ""]
    for name, _, _, cmds in summary:
        for k in ("trace", "fetch", "write", "sq"):
            lines.append("    " + cmds[k])
    lines += ["", "Copy calibration: as in step_e6_f32_128cube_traffic.txt.", ""]
    out = os.path.join(ROOT, "profiles", "step_e6_f32_128cube_designs.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print(open(out).read())


def cpu_baseline(L, R0, steps, steps_1t):
    """The FP64 oracle on the same workload, a bounded number of steps on all
    the host threads and a smaller number on one thread."""
    from oracle import oracle as O
    from paper_2112_02574_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def rate(nthreads, nsteps):
        o = O.Oracle(3, 6, (L, L, L), tau=1.0, g=G_SYM, nthreads=nthreads)
        # the oracle takes no input from the GPU library, so it starts from the
        # plain tanh droplet (1.0 / 0.04): the cost of a step does not depend on it
        o.set_density(*inputs.droplet(L, L, L, R=R0))
        o.run(1)  # first touch of the work arrays
        t0 = time.perf_counter()
        o.run(nsteps)
        return time.perf_counter() - t0

    dt = rate(threads, steps)
    out = {"value": round(L ** 3 * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
           "kind": "oracle",
           "sample": f"FP64 oracle, {steps} steps of a {L}^3 D3Q19/E6 droplet "
                     f"({L ** 3 * steps:.3g} site updates, {dt:.1f} s)"}
    if steps_1t > 0:
        dt1 = rate(1, steps_1t)
        out["value_1thread"] = round(L ** 3 * steps_1t / dt1 / 1e6, 3)
        out["sample_1thread"] = f"{steps_1t} steps on 1 thread ({dt1:.1f} s)"
    out["cpu"] = _cpu_model()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _timed(step, steps, stream):
    """Event-timed milliseconds per step of ``step(n)`` on ``stream``."""
    import torch
    step(min(20, steps))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    step(steps)
    ev1.record(stream)
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / steps


# bytes per site update (read + write every population once) by storage;
# node storage keeps the rest populations in FP32: 36 x 2 + 2 x 4 each way
STORAGE_BYTES = {"f64": 608, "f32": 304, "f16_offset": 152, "bf16_offset": 152,
                 "f16_node": 160, "bf16_node": 160}
PRECISION_JSON = os.path.join(ROOT, "profiles", "precision_256cube_asym.json")


def _storage_kinds(scmc):
    return (("f64", scmc.F64), ("f32", scmc.F32), ("f16_offset", scmc.F16_OFF),
            ("bf16_offset", scmc.BF16_OFF), ("f16_node", scmc.F16_NODE),
            ("bf16_node", scmc.BF16_NODE))


def _storage_rate(args, scmc, shape, g, storage, n0, init, dev, stream, bps):
    s = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, g=g, storage=storage, n0=n0),
                 device=dev, stream=stream)
    if storage != scmc.F64:
        s.scmc_autotune(args.tune_cache)
    s.scmc_set_density(*init)
    ms = _timed(s.scmc_step, args.variant_steps, stream)
    kernel, tile = s.scmc_config()
    s.close()
    N = shape[0] * shape[1] * shape[2]
    return {"MLUPS": round(N / (ms * 1e3), 1), "kernel": KERNEL_NAMES[kernel], "tile": list(tile),
            "bytes_per_site": bps, "hbm_frac": round(bps * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def variants(args, L, R0, bulk, init, dev, stream):
    """Step rates of the other storage formats on the same droplet; of the
    256^3 asymmetric workload (B-rich droplet, g_AA = -0.2) in every storage,
    each beside its R_s and sigma_s error against FP64 storage from the
    precision study (profiles/precision_256cube_asym.json, 61440 steps); and
    of the 48-member batched sweep, each over ``args.variant_steps`` timed
    steps."""
    from paper_2112_02574_amd import inputs
    from paper_2112_02574_amd import scmc
    n0 = (0.5 * (bulk[0] + bulk[2]), 0.5 * (bulk[1] + bulk[3]))
    out = {}
    for name, storage in _storage_kinds(scmc):
        if name == "f32":
            continue
        out[name] = _storage_rate(args, scmc, (L, L, L), G_SYM, storage, n0, init, dev, stream,
                                  STORAGE_BYTES[name])
    # the 256^3 asymmetric droplet: its moment field outgrows the caches, so
    # the moment two-pass runs in z-slabs
    bulk_asym, _ = scmc.scmc_flat_equilibrium(
        scmc.problem(scmc.D3Q19, scmc.E6, (128, 128, 128), g=G_ASYM, storage=scmc.F64),
        lx=128, guess=inputs.FLAT_GUESS[-0.2], tol=1e-10, device=dev, stream=stream)
    Lb = 2 * L
    init_b = inputs.droplet(Lb, Lb, Lb, R=Lb / 4, a_rich=False, bulk=bulk_asym)
    n0_b = (0.5 * (bulk_asym[0] + bulk_asym[2]), 0.5 * (bulk_asym[1] + bulk_asym[3]))
    acc = {}
    if os.path.exists(PRECISION_JSON):
        with open(PRECISION_JSON) as fh:
            acc = json.load(fh)
    c5 = {"workload": f"D3Q19 E6 {Lb}^3 B-rich droplet R0={Lb / 4:g} g_AB=1.8 g_AA=-0.2 psi=n",
          "accuracy_steps": acc.get("steps")}
    for name, storage in _storage_kinds(scmc):
        r = _storage_rate(args, scmc, (Lb, Lb, Lb), G_ASYM, storage, n0_b, init_b, dev, stream,
                          STORAGE_BYTES[name])
        a = acc.get("runs", {}).get(name, {})
        r["abs_err_R_s_vs_f64"] = a.get("abs_err_R_s")
        r["rel_err_sigma_s_vs_f64"] = a.get("rel_err_sigma_s")
        r["abs_err_R_s_shell_vs_f64"] = a.get("abs_err_R_s_shell")
        c5[name] = r
    out[f"asym_{Lb}cube"] = c5
    out["batch48_f32"] = _batch_rate(args, bulk, bulk_asym, dev, stream, args.variant_steps)
    out["steps_each"] = args.variant_steps
    return out


def _batch_rate(args, bulk, bulk_asym, dev, stream, steps, graph=64):
    """The batched sweep: 48 droplets on 48^3..160^3 boxes, symmetric and
    asymmetric couplings, FP32, the design the batch autotuner picks, graphs of
    ``graph`` steps (0: direct launches); step rate over ``steps`` timed
    steps."""
    from paper_2112_02574_amd import inputs
    from paper_2112_02574_amd import scmc
    members = inputs.batch_members()
    bulks = {0.0: bulk, -0.2: bulk_asym}
    ps = [scmc.problem(scmc.D3Q19, scmc.E6, (m["L"],) * 3, g=m["g"], storage=scmc.F32)
          for m in members]
    b = scmc.Batch(ps, device=dev, stream=stream)
    tile = b.scmc_batch_autotune(args.tune_cache)
    for i, m in enumerate(members):
        Lm = m["L"]
        b.scmc_batch_set_density(i, *inputs.droplet(Lm, Lm, Lm, R=m["R0"], a_rich=m["a_rich"],
                                                    bulk=bulks[m["g"][0][0]]))
    b.scmc_batch_set_graph_steps(graph)
    # untimed: the first run of `graph` steps captures and instantiates the
    # graph (72 launches per step), a one-time cost outside the step rate
    b.scmc_batch_step(max(graph, 1))
    ms = _timed(b.scmc_batch_step, steps, stream)
    sites = sum(m["L"] ** 3 for m in members)
    gbs = 4 * 19 * 4 * sites / (ms * 1e-3) / 1e9
    r = {"MLUPS": round(sites / (ms * 1e3), 1), "sites": sites, "members": len(members),
         "tile": list(tile), "grid": b.scmc_batch_config()[1], "graph_steps": graph,
         "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    b.close()
    return r


def batch_only(args):
    """Profiling mode: the batched sweep alone, 20 untimed and --steps timed
    steps, in direct launches unless --graph is given (rocprofv3's counter
    collection has crashed the process on graph-launched dispatches)."""
    import torch
    from paper_2112_02574_amd import inputs
    from paper_2112_02574_amd import scmc
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    bulk, _ = scmc.scmc_flat_equilibrium(
        scmc.problem(scmc.D3Q19, scmc.E6, (128, 128, 128), g=G_SYM, storage=scmc.F64),
        lx=128, guess=inputs.FLAT_GUESS[0.0], tol=1e-10, device=dev, stream=stream)
    bulk_asym, _ = scmc.scmc_flat_equilibrium(
        scmc.problem(scmc.D3Q19, scmc.E6, (128, 128, 128), g=G_ASYM, storage=scmc.F64),
        lx=128, guess=inputs.FLAT_GUESS[-0.2], tol=1e-10, device=dev, stream=stream)
    print(json.dumps({"batch48_f32": _batch_rate(args, bulk, bulk_asym, dev, stream, args.steps,
                                                 graph=args.graph)}), flush=True)


def run(args):
    import torch

    from paper_2112_02574_amd import inputs
    from paper_2112_02574_amd import scmc

    L, R0 = args.size, args.size * 24.0 / 128.0
    N = L ** 3
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    if args.init == "flat":
        # stage one of the initialisation: bulk values of a converged flat interface
        bulk, flat_steps = scmc.scmc_flat_equilibrium(
            scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), g=G_SYM, storage=scmc.F64),
            lx=L, guess=inputs.FLAT_GUESS[0.0], tol=1e-10, device=dev, stream=stream)
    else:
        bulk, flat_steps = list(inputs.FLAT_GUESS[0.0]), 0
    init = inputs.droplet(L, L, L, R=R0, bulk=bulk)
    storage = dict(_storage_kinds(scmc))[args.storage]
    n0 = (0.5 * (bulk[0] + bulk[2]), 0.5 * (bulk[1] + bulk[3]))
    p = scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), tau=1.0, g=G_SYM,
                     storage=storage, n0=n0, kernel=KERNELS[args.kernel],
                     tile=tuple(args.tile) if args.tile else (0, 0, 0))
    sim = scmc.Sim(p, device=dev, stream=stream)
    if args.tile is None and args.kernel == "auto":
        sim.scmc_autotune(args.tune_cache)   # picks design and tile on this GPU
    if args.graph:
        sim.scmc_set_graph_steps(args.graph)
    sim.scmc_set_density(*init)
    kernel, tile = sim.scmc_config()

    sim.scmc_step(args.warmup)
    sim.scmc_synchronize()
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    step_ms = 0.0
    obs = stats = conv = None

    def monitor():
        # monitoring reductions (FP64): statistics, pressure tensor, sigma[R], R_s
        # and the convergence criteria of Sec. 4 (Delta P change, du, centre)
        return (sim.scmc_stats_get(), sim.scmc_observables(scmc.OBS_DROPLET, R0),
                sim.scmc_convergence_check(R0))

    t0 = time.perf_counter()
    done, at = 0, args.warmup
    while done < args.steps:
        # the reductions run whenever the run's step count reaches a multiple
        # of 2^11 (Sec. 4's cadence), inside the timed region when it does
        chunk = min(OBS_EVERY - at % OBS_EVERY, args.steps - done)
        ev0.record(stream)
        sim.scmc_step(chunk)
        ev1.record(stream)
        ev1.synchronize()
        step_ms += ev0.elapsed_time(ev1)
        done += chunk
        at += chunk
        if at % OBS_EVERY == 0:
            stats, obs, conv = monitor()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if obs is None:  # a run shorter than the cadence: observables after timing
        stats, obs, conv = monitor()

    ms_per_step = wall * 1e3 / args.steps
    mlups = N * args.steps / wall / 1e6
    kernel_ms = step_ms / args.steps
    bps = STORAGE_BYTES[args.storage]
    bytes_alg = bps * N  # read + write of every population once (FP32: 2 x 19 x 4 B each way)
    achieved = bytes_alg / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(N) if args.storage == "f32" else None
    # the streaming half of the step without arithmetic, in the same buffers:
    # the bandwidth ceiling of any design that moves each population once
    # (it overwrites the state, so it runs after the observables)
    copy_bytes = 4 * 19 * {"f64": 8, "f32": 4}.get(args.storage, 2) * N
    copy_gbs = copy_bytes / (sim.scmc_pull_copy(200) * 1e-6) / 1e9
    line = {
        "metric": "MLUPS (2-component D3Q19 Shan-Chen step)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64"}.get(args.storage, "f32"),
        "data": "synthetic (tanh droplet between flat-interface bulk values, no dataset)",
        "config": {"workload": f"D3Q19 E6 droplet {L}^3 R0={R0:g} tau=1 g_AB=1.8 psi=n "
                               f"{args.storage.upper() if args.storage == 'f32' else args.storage} SoA",
                   "storage": args.storage,
                   "sites": N, "kernel": KERNEL_NAMES[kernel],
                   "tile": list(tile), "graph_steps": args.graph,
                   "reductions_every": OBS_EVERY, "parallelism": "single GPU",
                   # the per-site sums (n_J, momentum, force, the mass closure)
                   # accumulate FP32 values in FP64, order-free
                   "site_sums": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel_ms": round(kernel_ms, 5),
                     "bytes_per_site": bps,
                     "pull_copy_GBs": round(copy_gbs, 1),
                     "pull_copy_frac": round(copy_gbs / HBM_PEAK_GBS, 4),
                     "achieved_over_pull_copy": round(achieved / copy_gbs, 4)},
        "observables": {"dP": _finite(obs["dP"]), "R_s": _finite(obs["R_s"]),
                        "sigma_s": _finite(obs["sigma_s"]), "step": obs["step"],
                        "mass": stats["mass"].tolist(), "max_u": _finite(stats["max_u"]),
                        "init_bulk": [round(v, 12) for v in bulk], "flat_steps": flat_steps,
                        "dP_change": _finite(conv["dP_change"]), "du": _finite(conv["du"]),
                        "com_offset": _finite(conv["com_offset"]),
                        "converged": conv["converged"]},
    }
    sim.close()
    if args.variant_steps > 0:
        line["variants"] = variants(args, L, R0, bulk, init, dev, stream)
    if args.cpu_steps > 0:
        line["cpu_baseline"] = cpu_baseline(L, R0, args.cpu_steps, args.cpu_steps_1t)
    print(json.dumps(line), flush=True)


def precision_study(args, out_md):
    """256^3 D3Q19 / E6 B-rich droplet, R0 = 64, g_AB = 1.8, g_AA = -0.2, psi = n:
    the same run with populations stored in FP64, FP32, FP16 and BF16 offsets
    from the global n0 (rounded to nearest even, or stochastically) and FP16
    and BF16 offsets from the per-node reference (FP32 arithmetic for all but
    FP64), observables every 2^11 steps.
    FP64 storage stands in for the oracle at this size (its parity with the
    oracle is tested on smaller lattices); errors are stated against it."""
    import torch

    from paper_2112_02574_amd import inputs
    from paper_2112_02574_amd import scmc

    L, R0 = args.size, args.size / 4.0
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    bulk, flat_steps = scmc.scmc_flat_equilibrium(
        scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), g=G_ASYM, storage=scmc.F64),
        lx=128, guess=inputs.FLAT_GUESS[-0.2], tol=1e-10, device=dev, stream=stream)
    init = inputs.droplet(L, L, L, R=R0, a_rich=False, bulk=bulk)
    n0 = (0.5 * (bulk[0] + bulk[2]), 0.5 * (bulk[1] + bulk[3]))
    runs = {}
    for name, storage, rounding in (
            ("f64", scmc.F64, 0), ("f32", scmc.F32, 0),
            ("f16_offset", scmc.F16_OFF, scmc.ROUND_NEAREST),
            ("bf16_offset", scmc.BF16_OFF, scmc.ROUND_NEAREST),
            ("f16_offset_sr", scmc.F16_OFF, scmc.ROUND_STOCHASTIC),
            ("bf16_offset_sr", scmc.BF16_OFF, scmc.ROUND_STOCHASTIC),
            ("f16_node", scmc.F16_NODE, scmc.ROUND_NEAREST),
            ("bf16_node", scmc.BF16_NODE, scmc.ROUND_NEAREST)):
        sim = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), g=G_ASYM, storage=storage,
                                    n0=n0, rounding=rounding, seed=12345),
                       device=dev, stream=stream)
        if storage != scmc.F64:
            sim.scmc_autotune(args.tune_cache)
        sim.scmc_set_density(*init)
        hist, step_ms, done = [], 0.0, 0
        while done < args.steps:
            k = min(OBS_EVERY, args.steps - done)
            step_ms += _timed_chunk(sim.scmc_step, k, stream)
            done += k
            o = sim.scmc_observables(scmc.OBS_DROPLET, R0)
            osh = sim.scmc_observables(scmc.OBS_SHELL, R0)
            st = sim.scmc_stats_get()
            hist.append({"step": done, "dP": _finite(o["dP"]), "R_s": _finite(o["R_s"]),
                         "sigma_s": _finite(o["sigma_s"]), "R_s_shell": _finite(osh["R_s"]),
                         "sigma_s_shell": _finite(osh["sigma_s"]), "max_u": _finite(st["max_u"]),
                         "mass": st["mass"].tolist()})
            print(f"{name} step {done}: dP={o['dP']:.6g} R_s={o['R_s']:.6g} "
                  f"sigma_s={o['sigma_s']:.6g}", flush=True)
        nA, nB = sim.scmc_get_fields()
        kernel, tile = sim.scmc_config()
        runs[name] = {"hist": hist, "MLUPS": round(L ** 3 * done / (step_ms * 1e3), 1),
                      "kernel": KERNEL_NAMES[kernel], "tile": list(tile),
                      "axis_nA": nA[L // 2, L // 2, :].copy(), "axis_nB": nB[L // 2, L // 2, :].copy()}
        sim.close()
    ref = runs["f64"]
    lines = ["# Storage precision on a 256^3 asymmetric droplet", "",
             "D3Q19, E6, 256^3 periodic, B-rich droplet R0 = 64 between the flat-interface bulk "
             "values (flat stage on 128 x 5 x 5, FP64: nA_in, nB_in, nA_out, nB_out = %s), tau = 1, "
             "g_AB = 1.8, g_AA = -0.2, g_BB = 0, psi = n; n0 = %s (midpoints of the bulk values). "
             "%d steps per run, observables every 2^11 steps. FP64 storage is the reference "
             "(its parity with the oracle is tested on smaller lattices)." % (
                 [round(float(v), 9) for v in bulk], [round(float(v), 6) for v in n0],
                 args.steps), "",
             "Command (repository root, one MI355X):", "",
             "    python bench.py --precision profiles/precision_256cube_asym.md --size %d --steps %d"
             % (L, args.steps), "",
             "The last two columns evaluate R_s on the shell-averaged profiles (observable "
             "kind SHELL, a variant of the paper's axis line) of the same states, against "
             "FP64's shell value.", "",
             "| storage | design | MLUPS | dP | R_s | sigma_s | abs err R_s | rel err sigma_s | "
             "max abs err n on axis | R_s (shells) | abs err R_s (shells) |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    out = {"workload": f"D3Q19 E6 {L}^3 B-rich droplet R0={R0:g} g_AA=-0.2", "steps": args.steps,
           "bulk": bulk.tolist() if hasattr(bulk, "tolist") else list(bulk), "runs": {}}
    for name, r in runs.items():
        f = r["hist"][-1]
        g = ref["hist"][-1]
        eR = abs(f["R_s"] - g["R_s"]) if f["R_s"] is not None and g["R_s"] is not None else None
        es = (abs(f["sigma_s"] - g["sigma_s"]) / abs(g["sigma_s"])
              if f["sigma_s"] is not None and g["sigma_s"] else None)
        en = float(max(np.abs(r["axis_nA"] - ref["axis_nA"]).max(),
                       np.abs(r["axis_nB"] - ref["axis_nB"]).max()))
        eRs = (abs(f["R_s_shell"] - g["R_s_shell"])
               if f["R_s_shell"] is not None and g["R_s_shell"] is not None else None)
        lines.append("| %s | %s | %.0f | %s | %s | %s | %s | %s | %.3g | %s | %s |" % (
            name, r["kernel"], r["MLUPS"], _fmt(f["dP"], "%.8g"), _fmt(f["R_s"], "%.8g"),
            _fmt(f["sigma_s"], "%.8g"), _fmt(eR, "%.3g"), _fmt(es, "%.3g"), en,
            _fmt(f["R_s_shell"], "%.8g"), _fmt(eRs, "%.3g")))
        out["runs"][name] = {"MLUPS": r["MLUPS"], "kernel": r["kernel"], "final": f,
                             "abs_err_R_s": eR, "rel_err_sigma_s": es, "max_abs_err_n_axis": en,
                             "abs_err_R_s_shell": eRs}
    lines += ["", "History of R_s (every 2^11 steps):", "",
              "| step | " + " | ".join(runs) + " |", "|---|" + "---|" * len(runs)]
    for i, h in enumerate(ref["hist"]):
        lines.append("| %d | " % h["step"] + " | ".join(
            _fmt(runs[n]["hist"][i]["R_s"], "%.6g") for n in runs) + " |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(os.path.splitext(out_md)[0] + ".json", "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def paper_couplings(dGAB, dGc=0.4):
    """g = G c_s^2 of the paper's runs (Sec. 4): G c_s^2 = 0.5 between the
    components and the self couplings of eq. self_p around the critical
    G_c c_s^2 = -e^2/3 of psi = exp(-1/n)."""
    Gc = -math.e ** 2 / 3.0
    return ((Gc * (1 - dGc * (1 + dGAB)), 0.5), (0.5, Gc * (1 - dGc)))


def tolman_sweep(args, out_md):
    """The paper's Tolman analysis at reduced size: for each dG_AB a flat
    interface (127 x 5 x 5, FP64) gives the bulk values and sigma_0, then A-rich
    and B-rich droplets with R0 = L/4 on odd boxes run (FP32) until Delta P
    changes by less than 1e-5 over 2^11 steps; sigma_s = Delta P R_s / 2 at the
    signed curvature +-1/R_s goes into the fit of eq. sigma_c."""
    import torch  # noqa: F401  (loads the HIP runtime before the library)
    from paper_2112_02574_amd import inputs, scmc
    dgs = [float(v) for v in args.tolman_dg.split(",")]
    Ls = [int(v) for v in args.tolman_L.split(",")]
    psi = scmc.PSI_EXP_NEG_INV
    lines = ["# Tolman length on the paper's parameter set (psi = exp(-1/n), D3Q19 / E4)", "",
             "Command (repository root, one MI355X):", "",
             f"    python3 bench.py --tolman OUT_MD --tolman-dg {args.tolman_dg} --tolman-L {args.tolman_L}",
             "", "| dG_AB | L | droplet | steps | centre offset | Delta P | R_s | sigma_s / sigma_0 |",
             "|---|---|---|---|---|---|---|---|"]
    fits = []
    for dg in dgs:
        g = paper_couplings(dg)
        t0 = time.time()
        pf = scmc.problem(scmc.D3Q19, scmc.E4, (31, 31, 31), g=g, psi_self=psi, storage=scmc.F64)
        bulk, _ = scmc.scmc_flat_equilibrium(pf, lx=127, guess=(2.0, 0.05, 0.05, 2.0), tol=1e-11,
                                             max_steps=400000)
        fl = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E4, (5, 5, 127), g=g, psi_self=psi,
                                   storage=scmc.F64))
        x = np.arange(127)
        inside = (x >= 31) & (x < 95)
        fl.scmc_set_density(np.broadcast_to(np.where(inside, bulk[0], bulk[2]), (5, 5, 127)).copy(),
                            np.broadcast_to(np.where(inside, bulk[1], bulk[3]), (5, 5, 127)).copy())
        fl.scmc_step(100000)
        sigma0 = fl.scmc_observables(scmc.OBS_FLAT)["sigma0"]
        fl.close()
        print(f"dG_AB {dg}: bulk {np.round(bulk, 6).tolist()} sigma0 {sigma0:.6f} "
              f"({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
        curv, sig = [], []
        for L in Ls:
            for a_rich in (True, False):
                t0 = time.time()
                n0 = (0.5 * (bulk[0] + bulk[2]), 0.5 * (bulk[1] + bulk[3]))
                s = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E4, (L, L, L), g=g, psi_self=psi,
                                          storage=scmc.F32, n0=n0))
                s.scmc_set_density(*inputs.droplet(L, L, L, R=L / 4, a_rich=a_rich, bulk=bulk))
                try:
                    c = s.scmc_run_to_convergence(L / 4, dt=2048, max_steps=args.tolman_max_steps,
                                                  tol_dP=1e-5)
                    o = s.scmc_observables(scmc.OBS_DROPLET, L / 4)
                except scmc.ScmcError as e:
                    c, o = None, None
                    print(f"  L {L} a_rich {a_rich}: {e}", file=sys.stderr, flush=True)
                s.close()
                kind = "A-rich" if a_rich else "B-rich"
                if c is None or not c["converged"] or c["com_offset"] > 1e-3:
                    lines.append(f"| {dg:+.2f} | {L} | {kind} | — | — | — | — | not converged |")
                    continue
                curv.append((1.0 if a_rich else -1.0) / o["R_s"])
                sig.append(o["sigma_s"])
                lines.append(f"| {dg:+.2f} | {L} | {kind} | {c['step']} | {c['com_offset']:.0e} | "
                             f"{o['dP']:.6f} | {o['R_s']:.4f} | {o['sigma_s'] / sigma0:.5f} |")
                print(f"  L {L} {kind}: steps {c['step']} R_s {o['R_s']:.4f} "
                      f"sigma_s/sigma0 {o['sigma_s'] / sigma0:.5f} ({time.time() - t0:.1f} s)",
                      file=sys.stderr, flush=True)
        fit = scmc.scmc_curvature_fit(curv, sig) if len(curv) >= 3 else (float("nan"),) * 3
        fits.append((dg, sigma0, fit, len(curv)))
    lines += ["", "Fit of eq. sigma_c over the converged droplets (scmc_curvature_fit):", "",
              "| dG_AB | sigma_0 flat | sigma_0 fit | relative difference | delta (lu) | 2 kbar + k (lu^2) | points |",
              "|---|---|---|---|---|---|---|"]
    for dg, sigma0, (s0, d, k), n in fits:
        lines.append(f"| {dg:+.2f} | {sigma0:.6f} | {s0:.6f} | {abs(s0 / sigma0 - 1):.2e} | "
                     f"{d:+.4f} | {k:.3f} | {n} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _fmt(v, f):
    return f % v if v is not None else "-"


def _timed_chunk(step, k, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    step(k)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--graph", type=int, default=0,
                    help="steps per captured hipGraph (0: direct launches)")
    ap.add_argument("--tile", type=int, nargs=3, default=None)
    ap.add_argument("--kernel", choices=sorted(KERNELS), default="auto")
    ap.add_argument("--tune-cache", default=os.path.join(os.environ.get("TMPDIR", "/tmp"),
                                                         "scmc_autotune.txt"))
    ap.add_argument("--init", choices=("flat", "tanh"), default="flat",
                    help="droplet bulk values: converged flat interface (default) or the "
                         "plain 1.0 / 0.04 guess (no flat-interface run: used by the "
                         "counter passes, whose per-dispatch counts do not depend on it)")
    ap.add_argument("--variant-steps", type=int, default=300,
                    help="timed steps of each storage variant and of the batched sweep "
                         "(0 to skip)")
    ap.add_argument("--cpu-steps", type=int, default=200,
                    help="oracle steps of the CPU baseline on all threads (0 to skip)")
    ap.add_argument("--cpu-steps-1t", type=int, default=10,
                    help="oracle steps of the CPU baseline on one thread (0 to skip)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (torch copy_), the "
                         "reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--precision", metavar="OUT_MD", default=None,
                    help="only run the storage-precision study (256^3 asymmetric droplet; "
                         "use --size 256 --steps N) and write its summary to OUT_MD")
    ap.add_argument("--tolman", metavar="OUT_MD", default=None,
                    help="only run the Tolman-length sweep on the paper's parameter set and "
                         "write its summary to OUT_MD")
    ap.add_argument("--tolman-dg", default="-0.88,-0.44,0,0.44,0.88",
                    help="comma-separated asymmetry parameters dG_AB of the sweep")
    ap.add_argument("--tolman-L", default="31,47,63,95,127",
                    help="comma-separated odd box sizes of the sweep (R0 = L/4)")
    ap.add_argument("--tolman-max-steps", type=int, default=400000)
    ap.add_argument("--summarize", metavar="DIR", default=None,
                    help="only write the profiles/ summaries from rocprofv3 output in DIR")
    ap.add_argument("--summarize-designs", metavar="OUTDIR", default=None,
                    help="write profiles/step_e6_f32_128cube_designs.md from the outputs of "
                         "design_profile_commands under OUTDIR")
    ap.add_argument("--summarize-tags", default="f32",
                    help="comma-separated profiled workloads to summarize (" + ",".join(PROFILE_RUNS) + ")")
    ap.add_argument("--storage", choices=sorted(STORAGE_BYTES), default="f32",
                    help="storage of the timed 128^3 droplet (the benchmark line: f32)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only time the 48-member batched sweep over --steps steps (profiling)")
    args = ap.parse_args()
    if args.precision:
        precision_study(args, args.precision)
        return
    if args.summarize_designs:
        summarize_designs(args.summarize_designs, args.size)
        return
    if args.summarize:
        for tag in args.summarize_tags.split(","):
            summarize_profiles(args.summarize, tag, args.size)
        return
    if args.tolman:
        tolman_sweep(args, args.tolman)
        return
    if args.batch_only:
        batch_only(args)
        return
    if args.copy_calib:
        import torch
        n = args.copy_calib * (1 << 20)
        a = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": n, "launches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding "
              "(sweep members or z-slabs per GPU) is not part of this library", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-process, single-GPU", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
