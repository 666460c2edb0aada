"""Summarise rocprofv3 CSV output into the short text files kept under profiles/.

kernel-trace mode: per-kernel call count and mean/min/max duration from a
``--kernel-trace --stats -f csv`` run.

counters mode: issue-level counters of one kernel (mean per dispatch over the
last dispatches with the largest grid) from any number of ``--pmc`` runs, and
the VALU issue utilisation they imply: wave-level VALU instructions x 4 cycles
(a wave64 instruction occupies a 16-lane SIMD for 4 cycles; some instructions
issue faster, so the ratio can exceed 1 when the pipes are saturated) over the
SIMD-cycles
of the dispatch (GRBM_GUI_ACTIVE, summed over the 8 XCDs, over 8, times 1024
SIMDs).

traffic mode: HBM bytes per dispatch of one kernel from two ``--pmc`` runs
(FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same
counter reads for the library's streaming copy of a known size (copy probe), and
stamped with the sha256 of the kernel source the counters were taken on.
"""
import argparse
import csv
import hashlib
import os
import statistics


def _rows(path):
    for name in os.listdir(path):
        if name.endswith("counter_collection.csv"):
            return list(csv.DictReader(open(os.path.join(path, name))))
    raise SystemExit(f"no counter_collection.csv under {path}")


def _values(path, counter, name_has, largest_grid=True, last=0):
    rows = [r for r in _rows(path) if r["Counter_Name"] == counter and name_has in r["Kernel_Name"]]
    if not rows:
        raise SystemExit(f"no {counter} rows for {name_has!r} in {path}")
    if largest_grid:
        g = max(int(r["Grid_Size"]) for r in rows)
        rows = [r for r in rows if int(r["Grid_Size"]) == g]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    if last:
        rows = rows[-last:]
    return [float(r["Counter_Value"]) for r in rows]


def traffic(a):
    fetch = _values(a.fetch, "FETCH_SIZE", a.kernel, last=a.last)
    write = _values(a.write, "WRITE_SIZE", a.kernel, last=a.last)
    cf = statistics.mean(_values(a.copy_fetch, "FETCH_SIZE", "copy_kernel"))
    cw = statistics.mean(_values(a.copy_write, "WRITE_SIZE", "copy_kernel"))
    f_scale = a.copy_bytes / (cf * 1024.0)
    w_scale = a.copy_bytes / (cw * 1024.0)
    fb = statistics.mean(fetch) * 1024.0 * f_scale
    wb = statistics.mean(write) * 1024.0 * w_scale
    sha = hashlib.sha256(open(a.source, "rb").read()).hexdigest()
    lines = [
        f"# HBM traffic per dispatch of {a.kernel} ({a.workload})",
        "# commands:",
        *[f"#   {c}" for c in a.command],
        f"# copy probe: {a.copy_bytes} bytes read and written per dispatch; FETCH_SIZE read "
        f"{cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB per copy dispatch",
        f"# dispatches used: {len(fetch)} (FETCH) / {len(write)} (WRITE), largest grid only"
        + (f", the last {a.last} (the timed estimates)" if a.last else ""),
        f"kernel: {a.kernel}",
        f"kernel_source_sha256: {sha}",
        f"fetch_kib_raw_mean: {statistics.mean(fetch):.3f}",
        f"write_kib_raw_mean: {statistics.mean(write):.3f}",
        f"fetch_scale: {f_scale:.5f}",
        f"write_scale: {w_scale:.5f}",
        f"fetch_bytes_per_launch: {fb:.0f}",
        f"write_bytes_per_launch: {wb:.0f}",
    ]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(a):
    vals = {}
    for path in a.runs:
        names = sorted({r["Counter_Name"] for r in _rows(path)})
        for n in names:
            v = _values(path, n, a.kernel, last=a.last)
            vals[n] = statistics.mean(v)
    lines = [f"# Issue counters per dispatch of {a.kernel} ({a.workload})", "# commands:",
             *[f"#   {c}" for c in a.command],
             f"# mean over the last {a.last} largest-grid dispatches (the timed estimates)",
             f"kernel: {a.kernel}",
             f"kernel_source_sha256: {hashlib.sha256(open(a.source, 'rb').read()).hexdigest()}"]
    lines += [f"{n}: {vals[n]:.6g}" for n in sorted(vals)]
    if "GRBM_GUI_ACTIVE" in vals and "SQ_INSTS_VALU" in vals:
        cycles = vals["GRBM_GUI_ACTIVE"] / a.xcds
        cap = cycles * a.simds
        lines += [f"dispatch_cycles: {cycles:.6g}",
                  f"valu_issue_utilisation: {4.0 * vals['SQ_INSTS_VALU'] / cap:.4f}"]
        if "SQ_ACTIVE_INST_VALU" in vals:
            lines.append(f"valu_active_utilisation: {4.0 * vals['SQ_ACTIVE_INST_VALU'] / cap:.4f}")
        f32 = [vals.get(k) for k in ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32",
                                     "SQ_INSTS_VALU_MUL_F32")]
        if all(x is not None for x in f32):
            flops = 64.0 * (2.0 * f32[0] + f32[1] + f32[2])   # at most: every lane active
            lines.append(f"fp32_flop_upper_bound_per_dispatch: {flops:.6g}")
            lines.append(f"fp32_arith_share_of_valu: {sum(f32) / vals['SQ_INSTS_VALU']:.4f}")
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def kernel_trace(a):
    path = a.trace
    stats = [n for n in os.listdir(path) if n.endswith("kernel_stats.csv")]
    rows = list(csv.DictReader(open(os.path.join(path, stats[0]))))
    out = [f"# Kernel time summary ({a.workload})", "", "Command:", "", "```"]
    out += a.command + ["```", "", "| kernel | calls | mean ms | min ms | max ms | share |",
                        "|---|---|---|---|---|---|"]
    for r in rows[: a.top]:
        name = r["Name"].replace("(anonymous namespace)::", "")
        name = name.split("(")[0] if "(" in name else name
        out.append(f"| `{name[:70]}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | "
                   f"{float(r['Percentage']):.2f} % |")
    traces = [n for n in os.listdir(path) if n.endswith("kernel_trace.csv")]
    if traces and a.kernel:
        rows = [r for r in csv.DictReader(open(os.path.join(path, traces[0])))
                if a.kernel in r["Kernel_Name"]]
        if rows:
            def grid(r):
                return int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            g = max(grid(r) for r in rows)
            big = sorted((r for r in rows if a.any_grid or grid(r) == g),
                         key=lambda r: int(r["Start_Timestamp"]))
            if a.last:
                big = big[-a.last:]
            ms = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in big]
            which = f"the last {a.last} " if a.last else ""
            sel = "" if a.any_grid else f" with the largest grid ({g} work-items)"
            out += ["", f"`{a.kernel}`, {which}dispatches{sel}: "
                    f"{len(ms)}, mean {statistics.mean(ms):.3f} ms, min {min(ms):.3f} ms, "
                    f"max {max(ms):.3f} ms"]
    out += ["", *a.note]
    open(a.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    t.add_argument("--kernel", default="render_loss_kernel<false, false>")
    t.add_argument("--source", default=os.path.join(os.path.dirname(__file__), "csrc", "kernels.hip"))
    t.add_argument("--workload", default="")
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--last", type=int, default=0,
                   help="only the last N largest-grid dispatches (the timed ones)")
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--runs", nargs="+", required=True)
    c.add_argument("--kernel", default="render_loss_kernel<false, false>")
    c.add_argument("--workload", default="")
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--last", type=int, default=2)
    c.add_argument("--xcds", type=int, default=8)
    c.add_argument("--simds", type=int, default=1024)
    c.add_argument("--source", default=os.path.join(os.path.dirname(__file__), "csrc", "kernels.hip"))
    c.add_argument("--out", required=True)
    k = sub.add_parser("trace")
    k.add_argument("--trace", required=True)
    k.add_argument("--workload", default="")
    k.add_argument("--command", action="append", default=[])
    k.add_argument("--note", action="append", default=[])
    k.add_argument("--top", type=int, default=8)
    k.add_argument("--kernel", default="render_loss_kernel<false, false>",
                   help="also summarise this kernel's largest-grid dispatches")
    k.add_argument("--last", type=int, default=0,
                   help="only the last N of those dispatches (the timed ones)")
    k.add_argument("--any-grid", action="store_true",
                   help="take the kernel's dispatches of every grid size, not only the largest")
    k.add_argument("--out", required=True)
    a = ap.parse_args()
    {"traffic": traffic, "counters": counters, "trace": kernel_trace}[a.mode](a)


if __name__ == "__main__":
    main()
