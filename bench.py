"""Benchmark: shift x RHS solves per second of the shifted-COCG solver on one MI355X.

Default workload: the diamond tight-binding lattice of 8x8x8 conventional cells
(4096 atoms x 4 orbitals = 16384 rows, 278,528 stored entries), 256 shifts
eps in [-12, 8] with eta = 0.005, 256 unit right-hand sides e_0..e_255, every pair
solved to relative residual 1e-8 (iteration cap 40000), full solutions x_k,j written
to HBM.  A step is one complete solve of all 65,536 pairs with inputs resident on
the device.

Prints one JSON line with the metric, the roofline of the dominant kernel (the
deferred per-shift update, timed with HIP events on its stream) and the FP64 CPU
oracle timed on a bounded sample of the same workload.

Other workloads (--workload): `cubic` (16^3 lattice, 64 shifts, G_00 to 1e-10, the
latency-bound case), `hubbard` (extended Hubbard ring, 11,778,624 rows, 128 shifts,
one complex right-hand side) and `batch` (--problems disordered cubic lattices of
uneven size, 32 unit RHS each, 512 shifts eta = 0.002, FP32 directions, one batched
solve).  --variants prints, on stderr, the same diamond problem
at a reduced number of right-hand sides solved by the plain FP64 path (one rhs at a
time, shift vectors updated every iteration), by the blocked update, batched, and with
FP32 storage, with the error of each against the FP64 batched result.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6   # MI355X FP64 vector (256 CUs x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFS = 157.3  # MI355X FP32 vector (packed)
METRIC = "shift\u00d7RHS solves/sec to rel. residual 1e-8; SpMV achieved HBM GB/s vs peak"
UPDATE_KERNEL_SOURCES = ["flush.hip", "device_common.h", "scocg_internal.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="diamond",
                    choices=["diamond", "cubic", "hubbard", "batch", "krylov", "manybody", "gradient"])
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"],
                    help="default fp64 (fp32 storage for the batch workload)")
    ap.add_argument("--problems", type=int, default=8, help="lattices in the batch workload")
    ap.add_argument("--wave", type=int, default=8, help="lattices per batched solve in the batch workload")
    ap.add_argument("--update-form", default="auto", choices=["auto", "step", "expanded"],
                    help="deferred update: step form, or expanded (FP64 matrix cores); auto is the step form")
    ap.add_argument("--schedule", default="auto", choices=["auto", "serial", "overlap"],
                    help="deferred update in order with the seed iterations, or overlapped with the next block")
    ap.add_argument("--matrix-free", action="store_true",
                    help="hubbard workload: apply H from per-species hopping tables (hubbard_upload)")
    ap.add_argument("--sites", type=int, default=0, help="manybody workload: ring sites (default 14)")
    ap.add_argument("--electrons", type=int, default=0,
                    help="manybody workload: electrons per spin (default half filling)")
    ap.add_argument("--full-solutions", action="store_true",
                    help="manybody workload: spectra from full solution vectors instead of projected solves")
    ap.add_argument("--stored-ground-state", action="store_true",
                    help="manybody workload: ground state on the stored sector matrix instead of the operator")
    ap.add_argument("--window", type=int, default=0,
                    help="G_jj workloads (cubic, batch): shifts per rhs whose full directions are kept "
                         "(seed candidates); the others cost scalar work only.  0: all")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--nu", type=int, default=0,
                    help="krylov workload: recurrence steps (default: the iterations shifted COCG needs)")
    ap.add_argument("--shifts-per-wg", type=int, default=0)
    ap.add_argument("--n-rhs", type=int, default=0, help="default 256 (diamond), 32 per lattice (batch)")
    ap.add_argument("--n-shift", type=int, default=0)
    ap.add_argument("--max-iter", type=int, default=0)
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--columns", type=int, default=0,
                    help="gradient workload: orbital columns (default all 16384), in batches of --n-rhs (256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="diamond workload: skip the plain single-rhs reference and the matrix-free Hubbard record")
    ap.add_argument("--cpu-iters", type=int, default=8000)
    ap.add_argument("--variants", type=int, default=0,
                    help="also compare solver forms on the diamond problem with this many rhs (stderr)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 2 GiB device to device once (reference for the HBM byte counters)")
    ap.add_argument("--pmc-summary", nargs=6, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR",
                                                       "BENCH_JSON", "COMMANDS_TXT"),
                    help="write profiles/k_flush_<workload>_traffic.{json,md} from rocprofv3 counter runs")
    ap.add_argument("--pmc-hotpath-summary", nargs=6,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR", "BENCH_JSON", "COMMANDS_TXT"),
                    help="write profiles/hot_path_<workload>_traffic.{md,json} from rocprofv3 counter runs of "
                         "every kernel")
    ap.add_argument("--trace-summary", nargs=3, metavar=("STATS_DIR", "BENCH_JSON", "COMMAND_TXT"),
                    help="write profiles/kernels_<workload>_stats.md from a rocprofv3 --stats run")
    ap.add_argument("--clock-summary", nargs=3, metavar=("PMC_DIR", "BENCH_JSON", "COMMAND_TXT"),
                    help="write profiles/k_flush_<workload>_clock.md from a rocprofv3 run with "
                         "GRBM_GUI_ACTIVE and SQ_INSTS_VALU_FMA_F64")
    return ap.parse_args()


def update_kernel_digest():
    """sha1 over the sources the deferred-update kernel is compiled from."""
    import hashlib

    h = hashlib.sha1()
    for name in UPDATE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0802_0748_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def library_digest():
    """sha1 over every source the library is compiled from (the whole hot path's kernels)."""
    import hashlib

    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_0802_0748_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()


def measured_hot_path(workload, config):
    """HBM bytes of one whole solve (every kernel of the path) from the committed rocprofv3
    counter summary, if it was taken on this workload and the current library sources."""
    path = os.path.join(ROOT, "profiles", f"hot_path_{workload}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("library_sources_sha1") != library_digest() or rec.get("workload") != config:
        return None
    return rec


def measured_kernels(workload, config):
    """Per-kernel rates of the hot path from the committed rocprofv3 summaries of the current
    library sources on this workload: the average duration of each kernel in the benchmark's
    own (overlapped) schedule from the kernel trace, its memory-side bytes per launch from the
    FETCH_SIZE / WRITE_SIZE summary, and the ratio.  None if either summary is missing or stale."""
    recs = []
    for name in (f"kernels_{workload}_stats.json", f"hot_path_{workload}_traffic.json"):
        try:
            with open(os.path.join(ROOT, "profiles", name)) as f:
                recs.append(json.load(f))
        except (OSError, ValueError):
            return None
    trace, traffic = recs
    digest = library_digest()
    if any(r.get("library_sources_sha1") != digest or r.get("workload") != config for r in recs):
        return None
    avg = {k["kernel"]: k["avg_us"] for k in trace["kernels"]}
    out = []
    for k in traffic["kernels"]:
        if k["kernel"] not in avg or k["dispatches"] < 100:
            continue
        per = (k["read_bytes"] + k["write_bytes"]) / k["dispatches"]
        gbs = per / 1e3 / avg[k["kernel"]]
        out.append({"kernel": k["kernel"].replace("HIP_vector_type<double, 2u>", "double2"),
                    "avg_us": avg[k["kernel"]], "memory_side_bytes_per_launch": per, "achieved_gbs": gbs,
                    "frac_of_peak": gbs / HBM_PEAK_GBS})
    return out


def measured_traffic(workload, config=None, precision="fp64"):
    """HBM bytes per launch of the update kernel from the committed rocprofv3 counter
    summary, if it was taken on this workload, configuration and storage precision (the
    kernel instance it names) and on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"k_flush_{workload}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        digest = update_kernel_digest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha1") != digest:
        return None
    if config is not None and rec.get("workload") != config:
        return None
    if ("double" in rec.get("kernel", "")) != (precision == "fp64"):
        return None
    return rec.get("hbm_bytes_per_launch")


COPY_BYTES = 2 ** 31


def copy_bandwidth(torch, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of 2 GiB (read + write counted), best
    of `reps` timed with events on the current stream."""
    x = torch.ones(COPY_BYTES // 16, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del x, y
    torch.cuda.empty_cache()
    return 2 * COPY_BYTES / best / 1e9


def copy_calibration():
    """One device-to-device copy of 2 GiB: the HBM byte counters read on it give the factor
    from counter units to bytes."""
    import torch

    x = torch.ones(COPY_BYTES // 16, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(f"[bench] copied {COPY_BYTES} bytes", file=sys.stderr, flush=True)
    return 0


def _read_csv(path):
    import csv

    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find_csv(d, suffix):
    for root, _, files in os.walk(d):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _bench_line(path):
    with open(path) as f:
        for ln in f:
            ln = ln.strip()
            if ln.startswith("{"):
                return json.loads(ln)
    raise ValueError(f"no JSON line in {path}")


def _main_update_dispatches(rows):
    """Counter rows of the benchmark solve's update kernel: the k_flush instance with the most
    dispatches, restricted to its largest grid (the small warm-up solve has a smaller one)."""
    rows = [r for r in rows if "k_flush" in r["Kernel_Name"]]
    by_name = {}
    for r in rows:
        by_name.setdefault(r["Kernel_Name"], []).append(r)
    name, rs = max(by_name.items(), key=lambda kv: len(kv[1]))

    def grid(r):
        if r.get("Grid_Size"):
            return int(r["Grid_Size"])
        return int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])

    gmax = max(grid(r) for r in rs)
    return name, [r for r in rs if grid(r) == gmax]


def pmc_summary(args):
    fetch_dir, write_dir, cfetch_dir, cwrite_dir, bench_json, commands_txt = args.pmc_summary
    line = _bench_line(bench_json)
    algo = line["roofline"]["bytes_per_launch"]
    name, fr = _main_update_dispatches(_read_csv(_find_csv(fetch_dir, "counter_collection.csv")))
    _, wr = _main_update_dispatches(_read_csv(_find_csv(write_dir, "counter_collection.csv")))
    fetch_kib = sum(float(r["Counter_Value"]) for r in fr) / len(fr)
    write_kib = sum(float(r["Counter_Value"]) for r in wr) / len(wr)

    def copy_kib(d):
        rows = [r for r in _read_csv(_find_csv(d, "counter_collection.csv")) if "copyBuffer" in r["Kernel_Name"]]
        return max(float(r["Counter_Value"]) for r in rows)

    cf, cw = copy_kib(cfetch_dir), copy_kib(cwrite_dir)
    # a copy of COPY_BYTES reads and writes COPY_BYTES each
    fscale, wscale = COPY_BYTES / (cf * 1024), COPY_BYTES / (cw * 1024)
    rd, wb = fetch_kib * 1024 * fscale, write_kib * 1024 * wscale
    with open(commands_txt) as f:
        commands = [c.strip() for c in f if c.strip()]
    rec = {"kernel": name.split("(")[0].replace("void ", ""), "workload": line["config"]["workload"],
           "launches": len(fr), "fetch_kib_per_launch": fetch_kib, "write_kib_per_launch": write_kib,
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw, "fetch_scale": fscale,
                                "write_scale": wscale},
           "hbm_bytes_per_launch": rd + wb, "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wb,
           "algorithmic_bytes_per_launch": algo, "ratio": (rd + wb) / algo, "commands": commands,
           "kernel_sources_sha1": update_kernel_digest(),
           "kernel_sources": [f"paper_0802_0748_amd/csrc/{n}" for n in UPDATE_KERNEL_SOURCES]}
    out = os.path.join(ROOT, "profiles", f"k_flush_{args.workload}_traffic")
    with open(out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    cmd_block = "\n".join(commands)
    md = f"""# HBM traffic of the deferred per-shift update ({args.workload} workload)

Kernel `{rec['kernel']}`, {rec['workload']}. Counters per dispatch from two rocprofv3 runs, averaged
over the {len(fr)} launches of the benchmark solve (the small warm-up solve is excluded by grid size),
and a plain 2 GiB device copy for calibration (`bench.py --copy-calibration`):

```
{cmd_block}
```

| counter | copy of 2 GiB (KiB) | bytes per KiB | k_flush per launch (KiB) | k_flush per launch (GB) |
|---|---:|---:|---:|---:|
| FETCH_SIZE | {cf:.0f} | {fscale * 1024:.1f} | {fetch_kib:.0f} | {rd / 1e9:.2f} |
| WRITE_SIZE | {cw:.0f} | {wscale * 1024:.1f} | {write_kib:.0f} | {wb / 1e9:.2f} |

Measured HBM traffic per launch: **{(rd + wb) / 1e9:.2f} GB**; algorithmic bytes per launch (x_k and u_k read
and written once for every active pair, the residual history read once per rhs, counted on the device):
**{algo / 1e9:.2f} GB**; ratio {(rd + wb) / algo:.3f}.

Kernel sources: {', '.join(UPDATE_KERNEL_SOURCES)} (under paper_0802_0748_amd/csrc), sha1
`{rec['kernel_sources_sha1']}`; bench.py reports this traffic only while these sources are unchanged.
"""
    with open(out + ".md", "w") as f:
        f.write(md)
    print(f"[bench] wrote {out}.json/.md: {(rd + wb) / 1e9:.2f} GB per launch, ratio {(rd + wb) / algo:.3f}",
          file=sys.stderr)
    return 0


def pmc_hotpath_summary(args):
    """HBM traffic of the whole hot path: FETCH_SIZE and WRITE_SIZE summed over every dispatch of
    the benchmark run (all kernels), scaled by the same counters on a 2 GiB copy."""
    fetch_dir, write_dir, cfetch_dir, cwrite_dir, bench_json, commands_txt = args.pmc_hotpath_summary
    line = _bench_line(bench_json)

    def per_kernel(d):
        out = {}
        for r in _read_csv(_find_csv(d, "counter_collection.csv")):
            nm = r["Kernel_Name"].split("(")[0].replace("void ", "")
            c = out.setdefault(nm, [0, 0.0])
            c[0] += 1
            c[1] += float(r["Counter_Value"])
        return out

    def copy_kib(d):
        rows = [r for r in _read_csv(_find_csv(d, "counter_collection.csv")) if "copyBuffer" in r["Kernel_Name"]]
        return max(float(r["Counter_Value"]) for r in rows)

    fk, wk = per_kernel(fetch_dir), per_kernel(write_dir)
    cf, cw = copy_kib(cfetch_dir), copy_kib(cwrite_dir)
    fscale, wscale = COPY_BYTES / (cf * 1024), COPY_BYTES / (cw * 1024)
    names = sorted(set(fk) | set(wk), key=lambda n: -(fk.get(n, [0, 0])[1] * fscale + wk.get(n, [0, 0])[1] * wscale))
    kern = []
    for nm in names:
        rd = fk.get(nm, [0, 0.0])[1] * 1024 * fscale
        wr = wk.get(nm, [0, 0.0])[1] * 1024 * wscale
        kern.append({"kernel": nm, "dispatches": fk.get(nm, wk.get(nm, [0]))[0], "read_bytes": rd, "write_bytes": wr})
    total = sum(k["read_bytes"] + k["write_bytes"] for k in kern)
    with open(commands_txt) as f:
        commands = [c.strip() for c in f if c.strip()]
    steps = line["steps"]
    rec = {"workload": line["config"]["workload"], "steps": steps, "hbm_bytes_per_step": total / steps,
           "seconds_per_step": line["ms_per_step"] / 1e3, "kernels": kern,
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw},
           "commands": commands, "library_sources_sha1": library_digest()}
    out = os.path.join(ROOT, "profiles", f"hot_path_{args.workload}_traffic")
    with open(out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    write_hotpath_md(rec, out + ".md", args.workload)
    print(f"[bench] wrote {out}.json/.md: {total / steps / 1e9:.1f} GB per solve", file=sys.stderr)
    return 0


def write_hotpath_md(rec, path, workload):
    """The Markdown summary of a whole-path counter record (pmc_hotpath_summary)."""
    steps = rec["steps"]
    kern = rec["kernels"]
    total = rec["hbm_bytes_per_step"] * steps
    cf, cw = rec["copy_calibration"]["fetch_kib"], rec["copy_calibration"]["write_kib"]
    rows = "\n".join(f"| `{k['kernel'].replace('HIP_vector_type<double, 2u>', 'double2')}` | {k['dispatches']} | "
                     f"{k['read_bytes'] / steps / 1e9:.1f} | {k['write_bytes'] / steps / 1e9:.1f} |"
                     for k in kern[:12])
    cmd_block = "\n".join(rec["commands"])
    md = f"""# Memory traffic of the whole hot path ({workload} workload)

{rec['workload']}. FETCH_SIZE and WRITE_SIZE summed over every dispatch of the benchmark run (every
kernel of the path: seed iteration, shift scalars, deferred update, decisions), scaled by the same
counters on a plain 2 GiB device copy (FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB for 2 GiB read and
2 GiB written):

```
{cmd_block}
```

| kernel | dispatches | read GB per solve | written GB per solve |
|---|---:|---:|---:|
{rows}

Memory-side traffic per solve: **{total / steps / 1e9:.1f} GB**.  FETCH_SIZE and WRITE_SIZE count what the L2
caches fetch from and write back to the memory side, so Infinity Cache hits are included (the calibrating
copy is too large for that cache, so its scale is the HBM one).  The SpMV reads 5.7 times the bytes of its
direction vectors and matrix, as much as the matrix (3.3 MB) read once by each of the 128 groups of two
right-hand sides (428 MB per launch), which the Infinity Cache can hold.  Counter collection serialises and slows the kernels ({rec['seconds_per_step']:.2f} s for the
profiled solve), so bench.py divides these bytes by the solve time of its own run.  Library sources sha1
`{rec['library_sources_sha1']}`: bench.py reports this figure only while they are unchanged.
"""
    with open(path, "w") as f:
        f.write(md)


def trace_summary(args):
    stats_dir, bench_json, command_txt = args.trace_summary
    line = _bench_line(bench_json)
    rows = _read_csv(_find_csv(stats_dir, "kernel_stats.csv"))
    with open(command_txt) as f:
        command = f.read().strip()
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    wl = args.workload + ("_matrix_free" if args.matrix_free else "")
    out = os.path.join(ROOT, "profiles", f"kernels_{wl}_stats.md")
    lines = [f"# Kernel time, {wl.replace('_', ' ')} benchmark workload", "",
             f"{line['config']['workload']}; bench.py reported {line['value']:.1f} {line['unit']} "
             f"({line['ms_per_step'] / 1e3:.2f} s per solve) in this profiled run.", "",
             "```", command, "```", "",
             "| kernel | calls | total ms | average us | share |", "|---|---:|---:|---:|---:|"]
    for r in rows[:14]:
        nm = r["Name"].split("(")[0].replace("void ", "").replace("HIP_vector_type<double, 2u>", "double2")
        nm = nm.replace("HIP_vector_type<float, 2u>", "float2")
        lines.append(f"| `{nm}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} % |")
    try:
        trace = _read_csv(_find_csv(stats_dir, "kernel_trace.csv"))
    except FileNotFoundError:
        trace = []
    if trace and "avg_launch_ms" in line.get("roofline", {}):
        # the benchmark solve's update launches: the busiest k_flush instance at its largest grid
        name, disp = _main_update_dispatches(trace)
        avg_ms = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in disp) / len(disp) / 1e6
        lines += ["", f"Deferred update `{name.split('(')[0].replace('void ', '')}`: rocprofv3 average "
                      f"{avg_ms:.3f} ms per launch over the {len(disp)} launches of the benchmark solves; "
                      f"bench.py's HIP-event average over the same solves: {line['roofline']['avg_launch_ms']:.3f} ms "
                      f"({line['roofline']['bytes_per_launch'] / 1e9:.2f} GB and "
                      f"{line['roofline'].get('flops_per_launch', 0) / 1e9:.0f} GFLOP algorithmic per launch: "
                      f"{line['roofline']['achieved']:.1f} {line['roofline']['unit']}, "
                      f"{100 * line['roofline']['frac']:.1f} % of the {line['roofline']['bound']} peak)."]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    # the same rows as data, tied to the library sources, for the benchmark's per-kernel record
    rec = {"workload": line["config"]["workload"], "library_sources_sha1": library_digest(), "command": command,
           "kernels": [{"kernel": r["Name"].split("(")[0].replace("void ", ""), "calls": int(r["Calls"]),
                        "total_ms": float(r["TotalDurationNs"]) / 1e6, "avg_us": float(r["AverageNs"]) / 1e3}
                       for r in rows]}
    with open(out.replace(".md", ".json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"[bench] wrote {out}", file=sys.stderr)
    return 0


def clock_summary(args):
    """Engine clock and executed FP64 multiply-add rate of the update kernel, per dispatch
    from GRBM_GUI_ACTIVE (busy cycles, summed over the XCDs) and SQ_INSTS_VALU_FMA_F64 (wave
    instructions, 64 lanes x 2 flops each) over each dispatch's duration."""
    pmc_dir, bench_json, command_txt = args.clock_summary
    line = _bench_line(bench_json)
    with open(command_txt) as f:
        command = f.read().strip()
    agent = [r for r in _read_csv(_find_csv(pmc_dir, "agent_info.csv")) if r.get("Agent_Type") == "GPU"][0]
    n_xcc, n_cu = int(agent["Num_Xcc"]), int(agent["Cu_Count"])
    max_mhz = float(agent["Max_Engine_Clk_Fcompute"])
    name, rows = _main_update_dispatches(_read_csv(_find_csv(pmc_dir, "counter_collection.csv")))
    per = {}
    for r in rows:
        d = per.setdefault(int(r["Dispatch_Id"]), {})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    ids = sorted(per)
    q = max(1, (len(ids) + 3) // 4)
    parts = [("dispatches %d-%d" % (i, min(i + q, len(ids)) - 1), ids[i:i + q]) for i in range(0, len(ids), q)]
    parts.append(("all %d" % len(ids), ids))
    lines = [f"# Engine clock and FP64 rate of the deferred update ({args.workload} workload)", "",
             f"Kernel `{name.split('(')[0].replace('void ', '')}`, {line['config']['workload']}, update run alone "
             f"(serial schedule). Per dispatch: clock = GRBM_GUI_ACTIVE / {n_xcc} XCDs / duration; FP64 rate = "
             f"SQ_INSTS_VALU_FMA_F64 x 64 lanes x 2 flops / duration; peak = {n_cu} CUs x 128 flop/clk x clock.", "",
             "```", command, "```", "",
             "| dispatches | mean duration (ms) | clock (GHz) | executed FP64 (TFLOP/s) | of peak at "
             f"{max_mhz / 1e3:.1f} GHz | of peak at the measured clock |", "|---|---:|---:|---:|---:|---:|"]
    for label, sel in parts:
        ns = sum(per[i]["ns"] for i in sel)
        cyc = sum(per[i]["GRBM_GUI_ACTIVE"] for i in sel) / n_xcc
        fl = sum(per[i]["SQ_INSTS_VALU_FMA_F64"] for i in sel) * 64 * 2
        ghz = cyc / ns
        tfs = fl / ns / 1e3
        lines.append(f"| {label} | {ns / len(sel) / 1e6:.2f} | {ghz:.2f} | {tfs:.1f} | "
                     f"{100 * tfs / (n_cu * 128 * max_mhz / 1e6):.1f} % | {100 * tfs / (n_cu * 128 * ghz / 1e3):.1f} % |")
    out = os.path.join(ROOT, "profiles", f"k_flush_{args.workload}_clock.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"[bench] wrote {out}", file=sys.stderr)
    return 0


def cpu_baseline(p, gpu_iters, sample_iters, row_scale=None, converged=None):
    """Time the oracle on one right-hand side with all shifts for a fixed number of
    iterations (and with a single shift, to separate the seed cost), then scale to
    the whole workload with the per-pair iteration counts of the GPU solve (and, for
    right-hand sides of other sizes, by their row count relative to this one)."""
    from oracle import oracle as O

    b = p.rhs_dense()[0]
    O.shifted_cocg(p.H, p.z[:1], b, fixed_iter=2)  # load / warm
    t0 = time.perf_counter()
    O.shifted_cocg(p.H, p.z, b, fixed_iter=sample_iters, seed_index=0)
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.shifted_cocg(p.H, p.z[:1], b, fixed_iter=sample_iters, seed_index=0)
    t_one = time.perf_counter() - t0
    M = len(p.z)
    c_seed = t_one / sample_iters
    c_pair = max(t_all - t_one, 0.0) / ((M - 1) * sample_iters)
    scale = np.ones(gpu_iters.shape[0]) if row_scale is None else np.asarray(row_scale, dtype=float)
    seed_iters = gpu_iters.max(axis=1).sum()
    est = float(np.sum(scale * (c_seed * gpu_iters.max(axis=1) + c_pair * gpu_iters.sum(axis=1))))
    if converged is None:
        converged = gpu_iters.size
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the same sample on one thread, in a child process (the oracle's thread count is fixed
    # when it loads), a twentieth of the iterations
    single = None
    n1 = max(1, sample_iters // 20)
    code = ("import sys, time, numpy as np; sys.path.insert(0, sys.argv[1]); from oracle import oracle as O; "
            "from workloads import config1_cubic, config2_diamond, config3_hubbard; "
            "p = {'diamond': config2_diamond, 'cubic': config1_cubic}[sys.argv[2]](n_shift=int(sys.argv[3])); "
            "b = p.rhs_dense()[0]; O.shifted_cocg(p.H, p.z[:1], b, fixed_iter=2); n = int(sys.argv[4]); "
            "t0 = time.perf_counter(); O.shifted_cocg(p.H, p.z, b, fixed_iter=n, seed_index=0); "
            "t1 = time.perf_counter(); O.shifted_cocg(p.H, p.z[:1], b, fixed_iter=n, seed_index=0); "
            "print(t1 - t0, time.perf_counter() - t1)")
    wl = next((w for w in ("diamond", "cubic") if p.name.startswith(w)), None)
    if wl is not None and row_scale is None:
        import subprocess

        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code, ROOT, wl, str(M), str(n1)], env=env, capture_output=True,
                           text=True, timeout=600)
        if r.returncode == 0:
            a1, o1 = (float(v) for v in r.stdout.split())
            c1_seed, c1_pair = o1 / n1, max(a1 - o1, 0.0) / ((M - 1) * n1)
            est1 = float(np.sum(c1_seed * gpu_iters.max(axis=1) + c1_pair * gpu_iters.sum(axis=1)))
            single = dict(value=converged / est1, cores=1, sample=f"{n1} iterations ({a1:.1f} s, one shift {o1:.1f} s)")
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return dict(value=converged / est, unit="solves/s", cores=threads, kind="oracle", estimated=True,
                sample=(f"ESTIMATE, not an end-to-end run: oracle on the first rhs with all {M} shifts for "
                        f"{sample_iters} fixed iterations "
                        f"({t_all:.1f} s) and with one shift ({t_one:.1f} s); per-pair and per-seed iteration "
                        f"costs scaled by the GPU solve's iteration counts (sum {int(gpu_iters.sum())} pair-"
                        f"iterations, {int(seed_iters)} seed iterations) to an estimated {est:.3g} s"),
                single_thread=single, cpu_model=cpu_model, nproc=os.cpu_count())


def cpu_baseline_end_to_end(p, extrapolated):
    """The oracle as it stands, end to end on a bounded sample of the workload: the first
    right-hand side with every shift, solved to the workload's tolerance and cap on all host
    cores (OpenMP over the shifts), converged pairs over wall time.  The right-hand sides are
    alike (unit vectors of one matrix), so one of them is a fair sample; the per-iteration
    extrapolation to the whole workload is kept beside it."""
    from oracle import oracle as O

    b = p.rhs_dense()[0]
    O.shifted_cocg(p.H, p.z[:1], b, fixed_iter=2)  # load / warm
    t0 = time.perf_counter()
    out = O.shifted_cocg(p.H, p.z, b, tol=p.tol, max_iter=p.max_iter)
    t = time.perf_counter() - t0
    conv = int((out["status"] == 0).sum())
    return dict(value=conv / t, unit="solves/s", cores=extrapolated["cores"], kind="oracle",
                sample=(f"end to end: the oracle on the first of the {p.n_rhs} right-hand sides with all {len(p.z)} "
                        f"shifts to tol {p.tol:g} ({int(out['total_iters'])} iterations, {conv} pairs converged) in "
                        f"{t:.1f} s"),
                cpu_model=extrapolated["cpu_model"], nproc=extrapolated["nproc"], extrapolated=extrapolated)


def load_workload(args):
    from workloads import config1_cubic, config2_diamond, config3_hubbard

    if args.workload == "diamond":
        p = config2_diamond(n_shift=args.n_shift or 256, n_rhs=args.n_rhs or 256)
        p.max_iter, p.tol = 40000, 1e-8
        desc = (f"diamond 8x8x8 cells, 4 orbitals/atom (n={p.H.n}, nnz={p.H.nnz}), {len(p.z)} shifts eta=0.005, "
                f"{p.n_rhs} unit RHS")
    elif args.workload == "cubic":
        p = config1_cubic(n_shift=args.n_shift or 64)
        p.max_iter = 20000
        desc = f"simple cubic 16^3 (n={p.H.n}), {len(p.z)} shifts eta=0.01, G_00"
    else:
        p = config3_hubbard(n_shift=args.n_shift or 128)
        p.max_iter, p.tol = 20000, 1e-8
        desc = (f"extended Hubbard ring 14 sites 7+7 (n={p.H.n}, nnz={p.H.nnz}), {len(p.z)} shifts eta=0.05, "
                f"one complex unit RHS")
    if args.max_iter:
        p.max_iter = args.max_iter
    if args.tol:
        p.tol = args.tol
    return p, desc


def update_roofline(upd_ms, upd_bytes, upd_flops, upd_launches, workload, precision, config=None):
    """Roofline of the deferred per-shift update from its device-counted algorithmic bytes and
    flops over its summed launch time.  Its arithmetic intensity is about T * 16 flops per 64 B
    of x_k, u_k (FP64, T steps per block); above the machine balance (FP64 vector peak over
    HBM peak, 9.8 flop/B; FP32 storage: 19.7) the kernel is bound by its fused multiply-adds
    and is reported against the vector peak, below it against HBM."""
    t = upd_ms / 1e3
    gbs = (upd_bytes / 1e9) / t if t > 0 else 0.0
    tfs = (upd_flops / 1e12) / t if t > 0 else 0.0
    alu_peak = FP64_PEAK_TFS if precision == "fp64" else FP32_PEAK_TFS
    intensity = upd_flops / upd_bytes if upd_bytes > 0 else 0.0
    per = {"kernel": "k_flush (deferred per-shift update)", "avg_launch_ms": upd_ms / max(upd_launches, 1),
           "bytes_per_launch": upd_bytes / max(upd_launches, 1), "flops_per_launch": upd_flops / max(upd_launches, 1),
           "intensity_flop_per_byte": intensity, "hbm_achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
           "alu_achieved_tflops": tfs, "alu_frac": tfs / alu_peak}
    traffic = measured_traffic(workload, config, precision)
    if intensity > alu_peak * 1e3 / HBM_PEAK_GBS:
        return {"bound": "alu", "achieved": tfs, "peak": alu_peak, "unit": "TFLOP/s", "frac": tfs / alu_peak,
                "traffic": traffic, **per}
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, **per}


def hot_path(update_bytes, seed_iterations, n, elapsed, matrix_bytes=0, sweeps=0):
    """Whole hot path (seed SpMV and vector updates + deferred shift update) by a byte MODEL, not a
    measurement: the update kernel's device-counted bytes plus 8 complex FP64 vectors of n rows
    per seed iteration (p update: r, p read, p written; SpMV: p gathered, q written; residual: r,
    q read, r written) plus the stored matrix once per sweep of the batch, over the wall time of
    the timed solves.  The seed vectors largely stay in the 256 MB Infinity Cache, so these bytes
    overstate HBM traffic; the counter-measured figure is hot_path_measured."""
    nbytes = update_bytes + seed_iterations * 8 * 16 * n + matrix_bytes * sweeps
    gbs = nbytes / 1e9 / elapsed
    return {"model": "algorithmic bytes (seed vectors counted once per pass, cache hits included)",
            "achieved_gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "bytes": nbytes, "seconds": elapsed}


def bench_krylov(args, S, torch):
    """Krylov-subspace diagonalization (Sec. 3.2) of the diamond workload's local Green's
    functions G_jj(z_k), 256 unit RHS x 256 shifts, against shifted COCG on the same problem:
    COCG (projection mode, tol 1e-8) runs first as the reference and sets the step count nu to
    its iteration count; the Krylov method is then timed at nu and its largest deviation from
    the COCG G_jj reported (also at nu/4 and nu/2, on stderr).  Per recurrence step the
    algorithmic bytes are the seven passes over the real basis vectors (the matvec gathers K_n
    and reads K_{n-1}, writes K_n and w; the update reads both and writes w) plus the stored
    matrix once per group of four interleaved RHS."""
    from workloads import config2_diamond

    p = config2_diamond(n_rhs=args.n_rhs or 256)
    H = S.Hamiltonian.from_csr(p.H)
    K, M, n = p.n_rhs, len(p.z), p.H.n
    print(f"[bench] workload krylov: diamond n={n} nnz={p.H.nnz} shifts={M} rhs={K}", file=sys.stderr, flush=True)
    S.greens_diag(H, p.z[:4], p.rhs_idx[:1], fixed_iter=32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Gc, rep, _, rc = S.greens_diag(H, p.z, p.rhs_idx, tol=1e-8, max_iter=40000)
    torch.cuda.synchronize()
    t_cocg = time.perf_counter() - t0
    Gc = Gc.cpu().numpy()
    conv = rep["status"] == 0
    nu_cocg = int(rep["iters"].max())
    nu = args.nu or nu_cocg
    print(f"[bench] shifted COCG G_jj: {t_cocg:.2f} s rc={rc}, {int(conv.sum())}/{K * M} pairs at 1e-8, "
          f"{nu_cocg} iterations", file=sys.stderr, flush=True)

    def deviation(G):
        d = np.abs(G - Gc) / np.abs(Gc)
        return float(d[conv.T].max())

    for nu_s in sorted({max(1, nu // 4), max(1, nu // 2)}):
        G, _, _ = S.krylov_greens_diag(H, p.z, p.rhs_idx, nu_s)
        print(f"[bench] krylov nu={nu_s}: {S.last_timing()['total_ms'] / 1e3:.3f} s, max deviation from COCG "
              f"{deviation(G.cpu().numpy()):.2e}", file=sys.stderr, flush=True)
    S.krylov_greens_diag(H, p.z, p.rhs_idx[:4], 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_max, dev_ms = 0.0, 0.0
    for st in range(args.steps):
        G, ab, dim = S.krylov_greens_diag(H, p.z, p.rhs_idx, nu)
        dev_ms += S.last_timing()["total_ms"]
        dev_max = max(dev_max, deviation(G.cpu().numpy()))
        print(f"[bench] step {st}: krylov nu={nu} {S.last_timing()['total_ms'] / 1e3:.3f} s, max deviation "
              f"from COCG {dev_max:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    Kp = (K + 3) // 4 * 4
    step_bytes = 7 * 8 * n * Kp + 12 * int(p.H.nnz) * (Kp // 4)
    gbs = step_bytes * nu * args.steps / (dev_ms / 1e3) / 1e9
    line = {
        "metric": "shift\u00d7RHS local Green's functions/sec by Krylov-subspace diagonalization (nu steps); "
                  "max relative deviation from shifted COCG at 1e-8",
        "value": K * M * args.steps / elapsed, "unit": "G_jj(z)/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "diamond 8x8x8 cells, 4 orbitals/atom (n=16384, nnz=278528), 256 shifts "
                               "eta=0.005, 256 unit RHS, Krylov subspace diagonalization",
                   "n": n, "nnz": int(p.H.nnz), "n_shift": M, "n_rhs": K, "nu": nu},
        "accuracy": {"max_rel_deviation_from_cocg": dev_max, "cocg_seconds": t_cocg, "cocg_iterations": nu_cocg},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "three-term recurrence step",
                     "bytes_per_step": step_bytes, "us_per_step": dev_ms * 1e3 / (nu * args.steps),
                     "note": f"algorithmic bytes; the four basis-vector buffers ({4 * 8 * n * Kp / 1e6:.0f} MB) "
                             "fit the 256 MB Infinity Cache and the matrix re-reads hit L2, so part of "
                             "them never reaches HBM"},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = krylov_cpu_baseline(p, nu, K, M)
    return line


def krylov_cpu_baseline(p, nu, K, M):
    """The Krylov reference (numpy) on the first RHS for a sample of steps, scaled to K RHS x nu
    steps plus the subspace diagonalization per RHS."""
    from oracle import krylov as KR

    sample = min(nu, 2000)
    t0 = time.perf_counter()
    a, b = KR.lanczos(p.H, int(p.rhs_idx[0]), sample)
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    KR.greens_from_subspace(a, b, p.z)
    t_diag = time.perf_counter() - t0
    est = K * (t_rec * nu / sample + t_diag * (nu / sample) ** 3)
    return {"value": K * M / est, "unit": "G_jj(z)/s", "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "kind": "oracle",
            "sample": f"reference recurrence on the first rhs for {sample} steps ({t_rec:.1f} s) and its subspace "
                      f"diagonalization ({t_diag:.2f} s), scaled to {K} rhs x {nu} steps (diagonalization as "
                      f"nu^3) to an estimated {est:.3g} s"}


def bench_manybody(args, S, torch):
    """Ground state and single-particle spectrum (removal and addition) of the extended Hubbard
    ring (Sec. 2.2 and Sec. 4.2), by default 14 sites at half filling: the 7+7 sector
    (11,778,624 states, matrix-free operator) gets its ground state from 200 steps of the
    three-term recurrence and CG inverse iteration to ||H psi - E0 psi|| <= 1e-10;
    b = c_{0,up}|psi0> then lies in the 6+7 sector (10,306,296 states, matrix-free operator),
    where shifted COCG gives <b|((E0 - w) + i eta - H)^{-1}|b> at 128 energies w in [-10, 20],
    eta = 0.05 (removal spectrum; projected solves, Sec. 3.3); b' = c+_{0,up}|psi0> in the 8+7 sector gives the addition
    spectrum <b'|((E0 + w) + i eta - H)^{-1}|b'> the same way.  The removal weight <b|b> is the
    occupation <n_{0,up}> = N_up / L, and the two weights add up to exactly 1.  --sites and
    --electrons choose another sector (16 sites with 6 + 6 electrons has the 64,128,064 states
    of the paper's many-electron problem)."""
    from workloads import hubbard_ring

    L = args.sites or 14
    nu = nd = args.electrons or L // 2
    t0 = time.perf_counter()
    # the operator or the stored sector matrix (--stored-ground-state) give the same bits
    if args.stored_ground_state:
        H = S.Hamiltonian.from_csr(hubbard_ring(L, nu, nd, t=1.0, U=4.0, V=1.0))
    else:
        H = S.Hamiltonian.hubbard(L, nu, nd, t=1.0, U=4.0, V=1.0)
    form = "stored matrix" if args.stored_ground_state else "matrix-free operator"
    print(f"[bench] workload manybody: sector {nu}+{nd} of {L} sites, n={H.n} nnz={H.nnz} ({form}), built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    x0 = np.random.default_rng(0).normal(size=H.n)
    S.ground_state(S.Hamiltonian.from_csr(hubbard_ring(6, 3, 3)), np.ones(400), nu=20, tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psi, E0, E1, res, sweeps = S.ground_state(H, x0, nu=args.nu or 200, tol=1e-10)
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t0
    cg = S.last_timing()["iterations"] - 2 * (args.nu or 200)
    print(f"[bench] ground state: E0 {E0:.12f} (next estimate {E1:.6f}), residual {res:.1e}, {sweeps} sweeps, "
          f"{cg} CG iterations, {t_gs:.2f} s", file=sys.stderr, flush=True)
    M = args.n_shift or 128
    w = np.linspace(-10.0, 20.0, M)

    window = args.window or 32

    def spectrum(Hs, bv, z):
        """<b|(z_k - H)^{-1}|b> for all shifts: one projected solve (greens_proj) that carries
        every shift by scalars and keeps full directions for `window` seed candidates (--window,
        default 32).  With --full-solutions: full solutions, in one solve or in waves of shifts whose solution and
        direction vectors fit 200 GB beside the residual ring (shorter blocks for huge sectors,
        where the ring of 2T + 1 vectors would be large)."""
        if not args.full_solutions:
            Gw, rep, _, rc = S.greens_proj(Hs, z, bv[None, :], tol=1e-8, max_iter=20000, window=window)
            spectrum.iters = int(rep["iters"].max())
            return Gw[:, 0].cpu().numpy(), int((rep["status"] == 0).sum()), rc, 1
        n = Hs.n
        T = 48 if 97 * 16 * n < 64e9 else 16
        per_shift = 32 * n
        Mw = int(max(1, min(len(z), (200e9 - (2 * T + 1) * 16 * n) // per_shift)))
        G, conv, rc_all = [], 0, 0
        for k0 in range(0, len(z), Mw):
            X, rep, _, rc = S.shifted_cocg_solve(Hs, z[k0:k0 + Mw], bv[None, :], tol=1e-8, max_iter=20000, block=T)
            spectrum.iters = max(getattr(spectrum, "iters", 0), int(rep["iters"].max()))
            G.append((X[0] @ bv).cpu().numpy())
            conv += int((rep["status"] == 0).sum())
            rc_all = max(rc_all, rc)
            del X
            torch.cuda.empty_cache()
        return np.concatenate(G), conv, rc_all, (len(z) + Mw - 1) // Mw

    b, sec = S.hubbard_fermion_op(L, nu, nd, 0, 0, False, psi)
    Hm = S.Hamiltonian.hubbard(L, *sec, t=1.0, U=4.0, V=1.0)
    z = (E0 - w) + 0.05j
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G, conv, rc, nw = spectrum(Hm, b, z)
    torch.cuda.synchronize()
    t_sp = time.perf_counter() - t0
    # the same removal spectrum by Krylov-subspace diagonalization from b (Sec. 3.2): as many
    # steps of the recurrence as the shifted solve took iterations, then a continued fraction
    t0 = time.perf_counter()
    Gk, _, mk = S.krylov_greens_vec(Hm, z, b, spectrum.iters)
    torch.cuda.synchronize()
    t_kr = time.perf_counter() - t0
    dev_kr = float(np.max(np.abs(Gk.cpu().numpy() - G)) / np.max(np.abs(G)))
    print(f"[bench] removal spectrum by the continued fraction: {mk} steps, {t_kr:.2f} s, largest deviation "
          f"from shifted COCG {dev_kr:.1e} (relative to max |G|)", file=sys.stderr, flush=True)
    n_m = Hm.n
    del Hm, Gk
    A = -G.imag / np.pi
    occ = float((b.conj() @ b).real)  # total spectral weight <psi0|n_{0,up}|psi0>
    print(f"[bench] ionization spectrum: {M} energies ({nw} solve(s)), rc={rc}, {conv}/{M} converged, {t_sp:.2f} s; "
          f"total weight <b|b> {occ:.12f} (N_up/L = {nu / L:g}); peak at w = {w[np.argmax(A)]:.2f}",
          file=sys.stderr, flush=True)
    del b
    # the addition half: b' = c+_{0,up}|psi0> one up electron more, G+(w) = <b'|((E0 + w) + i eta - H)^{-1}|b'>
    bp, sec_p = S.hubbard_fermion_op(L, nu, nd, 0, 0, True, psi)
    del psi
    torch.cuda.empty_cache()
    Hp = S.Hamiltonian.hubbard(L, *sec_p, t=1.0, U=4.0, V=1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Gp, conv_p, rcp, nwp = spectrum(Hp, bp, (E0 + w) + 0.05j)
    torch.cuda.synchronize()
    t_ad = time.perf_counter() - t0
    Ap = -Gp.imag / np.pi
    occ_p = float((bp.conj() @ bp).real)
    print(f"[bench] affinity spectrum: {M} energies ({nwp} solve(s)), rc={rcp}, {conv_p}/{M} converged, {t_ad:.2f} s; "
          f"weight <b'|b'> {occ_p:.12f}; removal + addition weight {occ + occ_p:.15f} (exactly 1); "
          f"peak at w = {w[np.argmax(Ap)]:.2f}", file=sys.stderr, flush=True)
    return {
        "metric": "many-electron ground state (to residual 1e-10) and single-particle spectrum, removal and "
                  "addition (shift solves to rel. residual 1e-8), of the extended Hubbard ring",
        "value": (conv + conv_p) / (t_sp + t_ad), "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * (t_gs + t_sp + t_ad), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"extended Hubbard ring L={L}, t=1, U=4, V=1: ground state of {nu}+{nd} "
                               f"(n={H.n}, {form}), removal spectrum of c_(0,up) in {nu - 1}+{nd} (n={n_m}) and "
                               f"addition spectrum of c+_(0,up) in {nu + 1}+{nd} (n={Hp.n}), matrix-free, {M} "
                               "energies, eta=0.05" + (", full solutions" if args.full_solutions else
                                                       f", projected solves with {window} stored seed candidates"),
                   "n": int(H.n), "n_target": int(n_m),
                   "n_shift": M},
        "ground_state": {"E0": E0, "E1_estimate": E1, "residual": res, "sweeps": sweeps, "cg_iterations": int(cg),
                         "seconds": t_gs},
        "spectrum": {"seconds": t_sp, "converged": conv, "total_weight": occ, "occupation": nu / L,
                     "peak_w": float(w[np.argmax(A)])},
        "removal_by_continued_fraction": {"steps": mk, "seconds": t_kr, "max_rel_deviation_from_cocg": dev_kr},
        "addition_spectrum": {"seconds": t_ad, "converged": conv_p, "total_weight": occ_p,
                              "removal_plus_addition": occ + occ_p, "peak_w": float(w[np.argmax(Ap)])},
    }


def bench_batch(args, S, torch):
    """Disordered cubic lattices of uneven size (L in 24..64, W in {1, 4, 8}), 32 unit RHS per
    lattice, 512 shifts eta = 0.002, FP32 directions / FP64 scalars, all in one solve
    (greens_diag_batched: one seed SpMV and one update launch per block for every lattice)."""
    from workloads import config5_batch

    prec = args.precision or "fp32"
    probs = config5_batch(n_problems=args.problems, n_rhs=args.n_rhs or 32, n_shift=args.n_shift or 512)
    tol, max_iter = args.tol or 1e-8, args.max_iter or 80000
    Hs = [S.Hamiltonian.from_csr(p.H) for p in probs]
    z = probs[0].z
    rhs = [p.rhs_idx for p in probs]
    K = sum(len(r) for r in rhs)
    M = len(z)
    ntot = sum(p.H.n * len(p.rhs_idx) for p in probs)
    esz = 8 if prec == "fp32" else 16
    print(f"[bench] workload batch: {len(probs)} lattices L={[p.extra['L'] for p in probs]}, {K} rhs x {M} shifts, "
          f"{prec}; directions {M * ntot * esz / 1e9:.1f} GB", file=sys.stderr, flush=True)
    opts = dict(tol=tol, max_iter=max_iter, precision=prec, block=args.block, shifts_per_wg=args.shifts_per_wg,
                window=args.window, schedule=args.schedule)
    S.greens_diag_batched(Hs[:1], z[:4], [rhs[0][:1]], fixed_iter=32, precision=prec, block=args.block)
    torch.cuda.synchronize()
    S.set_profiling(True)
    upd_ms = upd_bytes = upd_flops = 0.0
    upd_launches = converged = 0
    iters = None
    t0 = time.perf_counter()
    # lattices go in waves of --wave lattices (one batched solve each)
    wave = max(1, args.wave)
    for st in range(args.steps):
        ts = time.perf_counter()
        status_l, iters_l, rcs = [], [], []
        for w0 in range(0, len(Hs), wave):
            tw = time.perf_counter()
            _, reps, rc = S.greens_diag_batched(Hs[w0:w0 + wave], z, rhs[w0:w0 + wave], **opts)
            t = S.last_timing()
            upd_ms += t["update_ms"]
            upd_bytes += t["update_bytes"]
            upd_flops += t["update_flops"]
            upd_launches += t["update_launches"]
            status_l += [r["status"] for r in reps]
            iters_l += [r["iters"] for r in reps]
            rcs.append(rc)
            ok = sum(int((r["status"] == 0).sum()) for r in reps)
            print(f"[bench] step {st} lattices {w0}..{min(w0 + wave, len(Hs)) - 1}: {time.perf_counter() - tw:.2f} s "
                  f"rc={rc} converged {ok} seed iterations {t['iterations']} blocks {t['blocks']}",
                  file=sys.stderr, flush=True)
        status = np.concatenate(status_l, axis=0)
        iters = np.concatenate(iters_l, axis=0)
        converged += int((status == 0).sum())
        ok_it = iters[status == 0]
        if ok_it.size:
            print(f"[bench] step {st}: iterations of converged pairs: median {int(np.median(ok_it))}, 90 % "
                  f"{int(np.percentile(ok_it, 90))}, 99 % {int(np.percentile(ok_it, 99))}, max {int(ok_it.max())}; "
                  f"unconverged {int((status != 0).sum())}", file=sys.stderr, flush=True)
        print(f"[bench] step {st}: {time.perf_counter() - ts:.2f} s rc={max(rcs)} converged "
              f"{int((status == 0).sum())}/{K * M}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    S.set_profiling(False)
    Ls = sorted(p.extra["L"] for p in probs)
    line = {
        "metric": METRIC, "value": converged / elapsed, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32-storage/f64-scalars", "data": "synthetic",
        "config": {"workload": (f"{len(probs)} disordered simple-cubic lattices L={Ls} (W in 1,4,8), "
                                f"{K} unit RHS ({len(rhs[0])} per lattice), {M} shifts eta=0.002, tol {tol:g}, "
                                f"max_iter {max_iter}, batched solves of {args.wave} lattices"
                                + (f", full directions for {args.window} seed candidates per rhs" if args.window
                                   else "")),
                   "n": int(sum(p.H.n for p in probs)), "nnz": int(sum(p.H.nnz for p in probs)), "n_shift": M,
                   "n_rhs": K, "precision": prec, "block": args.block or 48,
                   "iterations_per_step": int(np.max(iters))},
        "roofline": update_roofline(upd_ms, upd_bytes, upd_flops, upd_launches, "batch", prec, ""),
    }
    if not args.no_cpu_baseline:
        p0 = probs[0]
        sample = max(10, min(100000, int(args.cpu_iters * 4194304 / (M * p0.H.n))))
        scale = np.concatenate([[p.H.n / p0.H.n] * len(p.rhs_idx) for p in probs])
        line["cpu_baseline"] = cpu_baseline(p0, iters, sample, row_scale=scale,
                                            converged=int((status == 0).sum()))
    return line


def bench_gradient(args, S, torch):
    """Band energy, its gradient with respect to every stored entry of H and the forces on the
    atoms, on the 8x8x8 diamond cell (16384 orbitals): E = Re sum_q w_q z_q Tr G(z_q) over a
    128-node contour (Fermi level 0, the circle through the Gershgorin bound - 1), every orbital
    column solved by shifted COCG in batches of 256 right-hand sides (full solutions, whose
    pair products give dE/dH_ab), then forces -dE/dR through t(r) = exp(-2 (r - r0)) by torch
    autograd of the hopping values.  A step is the whole forward + gradient pass."""
    from paper_0802_0748_amd.autograd import hopping_values
    from workloads import config2_diamond
    from workloads.lattices import diamond_entry_map, diamond_geometry

    p = config2_diamond()
    Hc, geo = p.H, p.extra
    rows = np.repeat(np.arange(Hc.n), np.diff(Hc.row_ptr))
    diag = np.zeros(Hc.n)
    off = np.zeros(Hc.n)
    isd = rows == Hc.col
    diag[rows[isd]] = Hc.val[isd]
    np.add.at(off, rows[~isd], np.abs(Hc.val[~isd]))
    e_lo = float(np.min(diag - off)) - 1.0
    nq = args.n_shift or 128
    z, w = S.contour(e_lo, 0.0, nq)
    cols = np.arange(args.columns or Hc.n, dtype=np.int64)
    batch = args.n_rhs or 256
    tol, max_iter = args.tol or 1e-8, args.max_iter or 60000
    H = S.Hamiltonian.from_csr(Hc)
    kind, bond, o1, o2 = diamond_entry_map(Hc, geo["bonds"])
    _, bonds, vec0 = diamond_geometry(*geo["cells"])
    t_ = lambda a: torch.from_numpy(np.asarray(a))
    disp = t_(geo["displacement"].copy()).requires_grad_(True)
    vals = hopping_values(t_(vec0), disp, t_(bonds), t_(geo["blocks"]), t_(kind), t_(bond), t_(o1), t_(o2),
                          t_(Hc.val.copy()))
    assert np.max(np.abs(vals.detach().numpy() - Hc.val)) < 1e-12
    print(f"[bench] workload gradient: diamond n={Hc.n} nnz={Hc.nnz}, {nq}-node contour (min Im z "
          f"{z.imag.min():.4f}), {len(cols)} columns in batches of {batch}", file=sys.stderr, flush=True)
    S.density_matrix_energy(H, z[:4], w[:4], rhs_idx=cols[:2], want_grad=True, fixed_iter=32)
    torch.cuda.synchronize()
    S.set_profiling(True)
    upd_ms = upd_bytes = upd_flops = 0.0
    upd_launches = seed_iters = 0
    t0 = time.perf_counter()
    for st in range(args.steps):
        ts = time.perf_counter()
        E = 0.0
        dE = torch.zeros(Hc.nnz, dtype=torch.float64, device="cuda")
        for b0 in range(0, len(cols), batch):
            out = S.density_matrix_energy(H, z, w, rhs_idx=cols[b0:b0 + batch], want_rho=False, want_grad=True,
                                          tol=tol, max_iter=max_iter, allow_noconv=False)
            t = S.last_timing()
            upd_ms += t["update_ms"]
            upd_bytes += t["update_bytes"]
            upd_flops += t["update_flops"]
            upd_launches += t["update_launches"]
            seed_iters += t["iterations"]
            E += out["E"].item()
            dE += out["grad"]
            if (b0 // batch) % 8 == 0:
                print(f"[bench] step {st} columns {b0}..{b0 + batch - 1}: {time.perf_counter() - ts:.1f} s so far",
                      file=sys.stderr, flush=True)
        (g_disp,) = torch.autograd.grad(vals, disp, grad_outputs=dE.cpu())
        forces = -g_disp
        print(f"[bench] step {st}: {time.perf_counter() - ts:.2f} s, E = {E:.10f}, max |F| = "
              f"{forces.abs().max().item():.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    S.set_profiling(False)
    pairs = len(cols) * nq * args.steps
    line = {
        "metric": METRIC, "value": pairs / elapsed, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"band energy + dE/dH + forces, diamond 8x8x8 (n={Hc.n}, nnz={Hc.nnz}), "
                                f"{nq}-node contour with Fermi level 0, {len(cols)} orbital columns in batches of "
                                f"{batch}, tol {tol:g}, max_iter {max_iter}"),
                   "n": Hc.n, "nnz": int(Hc.nnz), "n_shift": nq, "n_rhs": int(len(cols)), "precision": "fp64",
                   "block": 48, "energy": E, "max_force": float(forces.abs().max())},
        "roofline": update_roofline(upd_ms, upd_bytes, upd_flops, upd_launches, "gradient", "fp64", ""),
    }
    return line


def plain_single_rhs(S, torch, H, p, B, value):
    """The plain FP64 GPU path on one right-hand side: the rhs alone, the shift vectors updated
    every iteration (block 1, step form), every shift to the tolerance.  The batched solve's
    speedup is stated against it (same tolerance, same FP64 arithmetic)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep, _, rc = S.shifted_cocg_solve(H, p.z, B[:1], tol=p.tol, max_iter=p.max_iter, block=1, update_form="step")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    conv = int((rep["status"] == 0).sum())
    rate = conv / t
    return {"value": rate, "unit": "solves/s", "seconds": t, "pairs": int(rep["status"].size), "converged": conv,
            "iterations": int(rep["iters"].max()), "speedup_of_value": value / rate,
            "note": "first rhs alone, FP64, shift vectors updated every iteration, same tolerance"}


def hubbard_matrix_free_record(S, torch, steps=1):
    """One solve of the extended Hubbard ring (14 sites, 7 + 7 electrons, 11,778,624 states; 128
    shifts eps in [-10, 20], eta = 0.05; one seeded unit complex rhs; tol 1e-8) on the matrix-free
    operator, with the deferred update's roofline: a second workload measured in the same run."""
    from workloads import config3_hubbard_rhs

    H = S.Hamiltonian.hubbard(14, 7, 7, t=1.0, U=4.0, V=1.0)
    z, b = config3_hubbard_rhs(0, H.n)
    B = torch.from_numpy(b[None, :]).cuda()
    M, n = len(z), H.n
    S.greens_proj(H, z[:4], B, fixed_iter=32)  # code paths for this operator (not timed)
    X = torch.empty((1, M, n), dtype=torch.complex128, device="cuda")
    S.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv = 0
    upd = [0.0, 0.0, 0.0, 0]
    for _ in range(steps):
        _, rep, _, rc = S.shifted_cocg_solve(H, z, B, out=X, tol=1e-8, max_iter=20000)
        t = S.last_timing()
        upd = [upd[0] + t["update_ms"], upd[1] + t["update_bytes"], upd[2] + t["update_flops"],
               upd[3] + t["update_launches"]]
        conv += int((rep["status"] == 0).sum())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.set_profiling(False)
    del X
    desc = (f"extended Hubbard ring 14 sites 7+7 (n={n}), matrix-free operator, {M} shifts eta=0.05, one complex "
            f"unit RHS, tol 1e-08, max_iter 20000")
    return {"metric": METRIC, "value": conv / el, "unit": "solves/s", "steps": steps, "ms_per_step": 1e3 * el / steps,
            "converged": conv, "dtype": "f64", "data": "synthetic",
            "config": {"workload": desc, "n": n, "n_shift": M, "n_rhs": 1, "iterations_per_step": int(rep["iters"].max())},
            "roofline": update_roofline(upd[0], upd[1], upd[2], upd[3], "hubbard_matrix_free", "fp64", desc)}


def cubic_record(S, torch, steps=3):
    """The small latency-bound workload: G_00(z_k) of the 16^3 simple-cubic lattice (on-site
    U[-1, 1], hopping -1), 64 shifts eps in [-7, 7] with eta = 0.01, tol 1e-10, projection mode;
    a third workload measured in the same run."""
    from workloads import config1_cubic

    p = config1_cubic()
    p.max_iter = 20000  # 1e-10 takes about 10,650 iterations, more than the stated 3,000
    H = S.Hamiltonian.from_csr(p.H)
    S.greens_diag(H, p.z[:4], p.rhs_idx, fixed_iter=32)  # code paths (not timed)

    def timed(tol):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        conv = 0
        for _ in range(steps):
            _, rep, _, rc = S.greens_diag(H, p.z, p.rhs_idx, tol=tol, max_iter=p.max_iter)
            conv += int((rep["status"] == 0).sum())
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return conv, el, int(rep["iters"].max())

    conv, el, it = timed(p.tol)
    conv8, el8, it8 = timed(1e-8)
    desc = f"simple cubic 16^3 (n={p.H.n}), 64 shifts eta=0.01, G_00, tol 1e-10, max_iter {p.max_iter}"
    return {"metric": METRIC, "value": conv / el, "unit": "solves/s", "steps": steps, "ms_per_step": 1e3 * el / steps,
            "converged": conv, "dtype": "f64", "data": "synthetic",
            "config": {"workload": desc, "n": p.H.n, "n_shift": len(p.z), "n_rhs": 1, "iterations_per_step": it},
            "at_tol_1e-8": {"value": conv8 / el8, "ms_per_step": 1e3 * el8 / steps, "converged": conv8,
                            "iterations_per_step": it8}}


def run_variants(S, torch, n_rhs):
    """The diamond problem with n_rhs right-hand sides solved by several forms of the solver."""
    from workloads import config2_diamond

    p = config2_diamond(n_rhs=n_rhs)
    H = S.Hamiltonian.from_csr(p.H)
    dev = torch.device("cuda")
    K, M, n = p.n_rhs, len(p.z), p.H.n
    B = torch.zeros((K, n), dtype=torch.complex128, device=dev)
    B[torch.arange(K), torch.from_numpy(p.rhs_idx).to(dev)] = 1.0
    base = dict(tol=1e-8, max_iter=40000)
    out = {}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    Xb, t_b = timed(lambda: S.shifted_cocg_solve(H, p.z, B, **base)[0])
    ref = Xb.cpu().numpy()
    out["batched fp64, block 48"] = (t_b, 0.0)
    forms = [("one rhs at a time, fp64, update every iteration (plain)", dict(block=1), 1),
             ("one rhs at a time, fp64, block 48", dict(block=48), 1),
             ("batched fp32 storage, block 48", dict(block=48, precision="fp32"), K),
             ("batched fp32 storage + fp64 refinement", dict(block=48, precision="fp32", refine=2), K)]
    for name, extra, per in forms:
        X = np.zeros_like(ref)
        t = 0.0
        for j0 in range(0, K, per):
            Xj, tj = timed(lambda: S.shifted_cocg_solve(H, p.z, B[j0:j0 + per], **base, **extra)[0])
            X[j0:j0 + per] = Xj.cpu().numpy()
            t += tj
        err = np.max(np.linalg.norm(X - ref, axis=2) / np.linalg.norm(ref, axis=2))
        out[name] = (t, err)
    print(f"[variants] diamond, {K} rhs x {M} shifts, tol 1e-8", file=sys.stderr)
    for name, (t, err) in out.items():
        print(f"[variants] {name:58s} {t:8.2f} s  {K * M / t:9.1f} solves/s  speedup vs plain "
              f"{out['one rhs at a time, fp64, update every iteration (plain)'][0] / t:6.2f}  max rel diff to "
              f"batched fp64 {err:.1e}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.pmc_summary:
        return pmc_summary(args)
    if args.trace_summary:
        return trace_summary(args)
    if args.pmc_hotpath_summary:
        return pmc_hotpath_summary(args)
    if args.clock_summary:
        return clock_summary(args)
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the solver runs on a "
              "single device and has no multi-GPU sharding.", file=sys.stderr)
        return 2
    import torch

    import paper_0802_0748_amd as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch":
        print(json.dumps(bench_batch(args, S, torch)), flush=True)
        return 0
    if args.workload == "krylov":
        print(json.dumps(bench_krylov(args, S, torch)), flush=True)
        return 0
    if args.workload == "manybody":
        print(json.dumps(bench_manybody(args, S, torch)), flush=True)
        return 0
    if args.workload == "gradient":
        print(json.dumps(bench_gradient(args, S, torch)), flush=True)
        return 0
    args.precision = args.precision or "fp64"
    p, desc = load_workload(args)
    if args.matrix_free:
        if args.workload != "hubbard":
            raise SystemExit("--matrix-free applies to the hubbard workload")
        e = p.extra
        H = S.Hamiltonian.hubbard(e["L"], e["n_up"], e["n_dn"], t=1.0, U=4.0, V=1.0)
        desc += ", matrix-free operator"
    else:
        H = S.Hamiltonian.from_csr(p.H)
    K, M, n = p.n_rhs, len(p.z), p.H.n
    greens = args.workload == "cubic"
    if not greens:
        B = torch.from_numpy(p.rhs_dense()).to(dev)
        X = torch.empty((K, M, n), dtype=torch.complex128, device=dev)
    opts = dict(tol=p.tol, max_iter=p.max_iter, precision=args.precision, block=args.block,
                shifts_per_wg=args.shifts_per_wg, schedule=args.schedule, update_form=args.update_form)
    if greens:
        opts["window"] = args.window
    elif args.window:
        raise SystemExit("--window applies to the G_jj workloads (cubic, batch)")

    def solve():
        if greens:
            return S.greens_diag(H, p.z, p.rhs_idx, **opts)
        return S.shifted_cocg_solve(H, p.z, B, out=X, **opts)

    print(f"[bench] workload {p.name}: n={n} nnz={p.H.nnz} shifts={M} rhs={K} {args.precision}", file=sys.stderr,
          flush=True)
    # initialise the library's code paths on a tiny problem (not a step)
    S.greens_diag(H, p.z[:4], p.rhs_idx[:1] if p.rhs_idx is not None else [0], fixed_iter=32, block=args.block,
                  precision=args.precision)
    torch.cuda.synchronize()
    S.set_profiling(True)
    for w in range(args.warmup):
        t0 = time.perf_counter()
        _, rep, _, rc = solve()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w}: {time.perf_counter() - t0:.2f} s rc={rc}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    upd_ms = upd_bytes = upd_flops = 0.0
    upd_launches = seed_iters = 0
    converged = 0
    iters = None
    t0 = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        _, rep, _, rc = solve()
        t = S.last_timing()
        upd_ms += t["update_ms"]
        upd_bytes += t["update_bytes"]
        upd_flops += t["update_flops"]
        upd_launches += t["update_launches"]
        seed_iters += t["iterations"]
        converged += int((rep["status"] == 0).sum())
        iters = rep["iters"]
        print(f"[bench] step {s}: {time.perf_counter() - ts:.2f} s rc={rc} converged "
              f"{int((rep['status'] == 0).sum())}/{K * M} seed iterations {t['iterations']} "
              f"blocks {t['blocks']} switches {t['switches']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    S.set_profiling(False)
    value = converged / elapsed
    wl_desc = (f"{desc}, tol {p.tol:g}, max_iter {p.max_iter}"
               + (f", full directions for {args.window} seed candidates" if args.window else ""))
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-storage/f64-scalars",
        "data": "synthetic",
        "config": {"workload": wl_desc,
                   "n": n, "nnz": int(p.H.nnz), "n_shift": M, "n_rhs": K, "precision": args.precision,
                   "block": args.block or 48, "schedule": args.schedule, "iterations_per_step": int(np.max(iters))},
        "roofline": update_roofline(upd_ms, upd_bytes, upd_flops, upd_launches, args.workload, args.precision,
                                    wl_desc if (args.block in (0, 48) and not args.shifts_per_wg) else ""),
        "hot_path": hot_path(upd_bytes, seed_iters, n, elapsed, 0 if args.matrix_free else 12 * int(p.H.nnz),
                             args.steps * int(np.max(iters))),
    }
    if args.precision == "fp32" and args.workload == "diamond":
        # FP32 storage on this problem ends about 34,000 iterations of rounding away from the
        # FP64 result (max relative deviation 5.7e-5), outside the 1e-5 wanted of it; at equal
        # accuracy the FP64 form is the faster one (FP32 + FP64 refinement costs 21 times more).
        line["accuracy_note"] = ("fp32 storage misses 1e-5 relative to fp64 on this workload "
                                 "(5.7e-5 measured); not competitive at equal accuracy")
    # achievable HBM bandwidth beside the 8 TB/s peak, measured after the timed region
    copy_gbs = copy_bandwidth(torch)
    line["hbm_copy"] = {"gbs": copy_gbs, "note": "device-to-device copy of 2 GiB, read + write counted"}
    line["hot_path"]["frac_of_copy"] = line["hot_path"]["achieved_gbs"] / copy_gbs
    rec = measured_hot_path(args.workload, wl_desc)
    if rec is not None:
        gbs = rec["hbm_bytes_per_step"] / 1e9 / (elapsed / args.steps)
        line["hot_path_measured"] = {"bound": "memory side of L2 (HBM, Infinity Cache hits included)",
                                     "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": gbs / HBM_PEAK_GBS, "frac_of_copy": gbs / copy_gbs,
                                     "hbm_bytes_per_step": rec["hbm_bytes_per_step"],
                                     "source": f"profiles/hot_path_{args.workload}_traffic.md (FETCH_SIZE + WRITE_SIZE "
                                               "over every kernel of one solve)"}
    kern = measured_kernels(args.workload, wl_desc)
    if kern is not None:
        # the SpMV and the other kernels of the path, each against the HBM peak (memory side of L2:
        # Infinity Cache hits included), from the committed trace and counter summaries
        line["kernels_measured"] = {"source": f"profiles/kernels_{args.workload}_stats.json (rocprofv3 kernel trace) "
                                              f"and profiles/hot_path_{args.workload}_traffic.json (FETCH_SIZE + "
                                              "WRITE_SIZE)", "peak_gbs": HBM_PEAK_GBS, "kernels": kern}
    if line["roofline"]["bound"] == "hbm":
        line["roofline"]["frac_of_copy"] = line["roofline"]["achieved"] / copy_gbs
    else:
        line["roofline"]["hbm_frac_of_copy"] = line["roofline"]["hbm_achieved_gbs"] / copy_gbs
    if not args.no_cpu_baseline:
        # the oracle's cost per iteration grows with shifts x rows: keep the sample near
        # --cpu-iters iterations of the diamond problem (256 x 16384)
        sample = max(10, min(100000, int(args.cpu_iters * 4194304 / (M * n))))
        line["cpu_baseline"] = cpu_baseline(p, iters, sample)
        if args.workload in ("diamond", "cubic"):
            line["cpu_baseline"] = cpu_baseline_end_to_end(p, line["cpu_baseline"])
    if args.workload == "diamond" and not args.no_extra and not greens:
        line["plain_single_rhs"] = plain_single_rhs(S, torch, H, p, B, value)
        print(f"[bench] plain single-rhs path: {line['plain_single_rhs']['seconds']:.2f} s for one rhs, batched speedup "
              f"{line['plain_single_rhs']['speedup_of_value']:.1f}", file=sys.stderr, flush=True)
        del X
        line["extra_workloads"] = {"hubbard_matrix_free": hubbard_matrix_free_record(S, torch),
                                   "cubic": cubic_record(S, torch)}
        print(f"[bench] matrix-free Hubbard: {line['extra_workloads']['hubbard_matrix_free']['ms_per_step'] / 1e3:.2f} s "
              "per solve", file=sys.stderr, flush=True)
    if args.variants:
        run_variants(S, torch, args.variants)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
