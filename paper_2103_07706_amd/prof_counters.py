"""HBM traffic of a kernel from rocprofv3 counter runs, calibrated by a copy.

Two steps:

1. On the GPU, four counter runs (one counter set per run), e.g. for the
   Jacobi Chebyshev step of the level-6 averaged right-hand side:

       rocprofv3 --pmc FETCH_SIZE --kernel-include-regex k_cheb_iter \\
           -f csv -d OUT/fetch -o run -- python3 bench.py --forms fp32_refined \\
           --tune-cache OUT/tune.json --graph 0 --steps 1 --warmup 0 --cpu-baseline 0
       (the same with WRITE_SIZE into OUT/write)
       rocprofv3 --pmc FETCH_SIZE -f csv -d OUT/copy_fetch -o run -- \\
           python3 -m paper_2103_07706_amd.prof_counters copy
       (the same with WRITE_SIZE into OUT/copy_write)

   `copy` runs one device-to-device copy of COPY_BYTES (plain streaming read
   and write of known size).

2. On any machine: `summarize` reads the four counter files and writes the
   per-launch HBM bytes of the kernel (FETCH_SIZE and WRITE_SIZE, each
   scaled by known bytes / counted bytes of the copy) as JSON, with a short
   markdown summary beside it.

`trace` summarises a `rocprofv3 --kernel-trace --stats -f csv` run of
bench.py: the per-kernel statistics of the whole run, and the average
duration of the bench's own timed launches of its roofline kernel (the last
`launches` dispatches of that kernel, the bench's final pass), next to the
average the bench measured with its per-launch events.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

COPY_BYTES = 1 << 30  # bytes read (and written) by the calibration copy
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_copy():
    import torch
    n = COPY_BYTES // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {COPY_BYTES} bytes", flush=True)


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        out += list(csv.DictReader(open(f)))
    return out


def per_dispatch(d, counter, name_filter=None):
    """Counter value (KiB, as rocprofv3 reports these derived counters) per
    dispatch, summed over the counter's instances; name_filter keeps the
    dispatches whose bare kernel name (kernel_base) is exactly it."""
    acc = {}
    for r in _rows(d):
        if r.get("Counter_Name") != counter:
            continue
        kn = r.get("Kernel_Name", "")
        if name_filter and kernel_base(kn) != name_filter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    return list(acc.values())


def kernel_source_hash(kernel="k_cheb_fused"):
    """Hash of the HIP source that defines the kernel."""
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2103_07706_amd", "csrc", "*.hip")))
    src = next((f for f in srcs if f" {kernel}(" in open(f).read()),
               os.path.join(ROOT, "paper_2103_07706_amd", "csrc", "pa_kernels.hip"))
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def summarize(a):
    fetch = per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
    write = per_dispatch(a.write, "WRITE_SIZE", a.kernel)
    cf = per_dispatch(a.copy_fetch, "FETCH_SIZE")
    cw = per_dispatch(a.copy_write, "WRITE_SIZE")
    if not (fetch and write and cf and cw):
        raise SystemExit("missing counter values")
    # the copy is the largest dispatch of its runs
    f_fetch = COPY_BYTES / (max(cf) * 1024.0)
    f_write = COPY_BYTES / (max(cw) * 1024.0)
    fb = statistics.mean(fetch) * 1024.0 * f_fetch
    wb = statistics.mean(write) * 1024.0 * f_write
    rec = {"kernel": a.kernel, "workload": a.workload, "backward": a.backward, "form": a.form,
           "kernel_source_sha256_16": kernel_source_hash(a.kernel),
           "dispatches": len(fetch), "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
           "hbm_bytes_per_launch": fb + wb,
           "copy_calibration": {"bytes_each_way": COPY_BYTES,
                                "fetch_kib_counted": max(cf), "write_kib_counted": max(cw),
                                "fetch_factor": f_fetch, "write_factor": f_write},
           "commands": a.commands}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    md = os.path.splitext(a.out)[0] + ".md"
    with open(md, "w") as f:
        f.write(f"# HBM traffic of {a.kernel}, workload {a.workload} ({a.backward} backward, "
                f"{a.form} form)\n\n")
        f.write("Counter runs (rocprofv3, one counter per run, from the repository root on the "
                "GPU machine):\n\n```\n" + "\n".join(a.commands) + "\n```\n\n")
        f.write(f"Copy calibration: {COPY_BYTES} bytes read and written; FETCH_SIZE counted "
                f"{max(cf):.0f} KiB (factor {f_fetch:.4f}), WRITE_SIZE {max(cw):.0f} KiB "
                f"(factor {f_write:.4f}).\n\n")
        f.write(f"{a.kernel}: {len(fetch)} dispatches; per launch, calibrated: fetch "
                f"{fb / 1e6:.3f} MB, write {wb / 1e6:.3f} MB, total {(fb + wb) / 1e6:.3f} MB.\n")
    print(json.dumps(rec, indent=1))


def kernel_base(name):
    """Bare kernel name: namespace, template arguments and parameters dropped."""
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0].split("<")[0].split("::")[-1]


def trace(a):
    def one(pattern):
        f = glob.glob(os.path.join(a.dir, "**", pattern), recursive=True)
        if not f:
            raise SystemExit(f"no {pattern} under {a.dir}")
        return list(csv.DictReader(open(f[0])))
    stats = one("*kernel_stats.csv")
    tr = one("*kernel_trace.csv")
    tr.sort(key=lambda x: int(x["Start_Timestamp"]))
    bench = None
    for line in open(a.bench_log):
        line = line.strip()
        if line.startswith("{") and '"roofline"' in line:
            bench = json.loads(line)
    if bench is None:
        raise SystemExit("no bench JSON line in " + a.bench_log)
    roof = bench["roofline"]
    plain = json.load(open(a.bench_json)) if a.bench_json else None
    k = roof["kernel"]
    mine = [x for x in tr if kernel_base(x["Kernel_Name"]) == k]
    last = mine[-int(roof["launches"]):]
    dur = [(int(x["End_Timestamp"]) - int(x["Start_Timestamp"])) / 1e3 for x in last]
    avg_us = sum(dur) / len(dur)
    with open(a.out, "w") as f:
        f.write(f"# Kernel trace: {bench['config']['workload']}, roofline kernel {k}\n\n")
        f.write("Command (from the repository root on the GPU machine):\n\n```\n" + a.command + "\n```\n\n")
        f.write("## Whole run (rocprofv3 --stats, every dispatch: set-up, autotuning and all forms)\n\n")
        f.write("| kernel | calls | total ms | avg us | % |\n|---|---|---|---|---|\n")
        for x in stats[:14]:
            f.write(f"| {kernel_base(x['Name'])} | {x['Calls']} | {float(x['TotalDurationNs']) / 1e6:.2f} | "
                    f"{float(x['AverageNs']) / 1e3:.2f} | {float(x['Percentage']):.1f} |\n")
        f.write(f"\n## The bench's timed launches of {k}\n\n")
        f.write(f"The last {len(last)} dispatches of {k} in the trace (the bench's final pass over "
                f"{bench['steps']} evaluations of its {bench['config'].get('form', '')} form): "
                f"average {avg_us:.2f} us per launch (min {min(dur):.2f}, max {max(dur):.2f}).\n\n")
        bpl = roof["algorithmic_bytes_per_launch"]
        f.write(f"Algorithmic bytes per launch {bpl / 1e6:.3f} MB: at the traced duration "
                f"{bpl / (avg_us * 1e-6) / 1e9:.0f} GB/s = {100 * bpl / (avg_us * 1e-6) / 1e9 / roof['peak']:.1f}% "
                f"of {roof['peak']:.0f} GB/s.\n\n")
        f.write("Under the profiler the bench's own event spans include the profiler's gaps "
                f"between dispatches ({roof['avg_launch_us']:.2f} us per launch in this run); "
                "they are not comparable with kernel durations.\n\n")
        if plain:
            pr = plain["roofline"]
            f.write(f"The same bench without the profiler ({plain['config'].get('form', '')} form "
                    f"timed, {pr['kernel']}): {pr['avg_launch_us']:.2f} us per launch over "
                    f"{pr['launches']} launches (ratio to the traced kernel average "
                    f"{pr['avg_launch_us'] / avg_us:.3f}), {pr['achieved']:.0f} GB/s = "
                    f"{100 * pr['frac']:.1f}% of peak; value {plain['value']:.2f} {plain['unit']}, "
                    f"{plain['ms_per_step']:.3f} ms per step.\n")
    print(open(a.out).read())


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    t = sub.add_parser("trace")
    t.add_argument("--dir", required=True)
    t.add_argument("--bench-log", dest="bench_log", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--bench-json", dest="bench_json", default=None,
                   help="JSON line of the same bench run without the profiler")
    s = sub.add_parser("summarize")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernel", "workload", "backward", "form",
              "out"):
        s.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    s.add_argument("--command", dest="commands", action="append", default=[])
    a = ap.parse_args()
    if a.cmd == "copy":
        run_copy()
    elif a.cmd == "trace":
        trace(a)
    else:
        summarize(a)


if __name__ == "__main__":
    main()
