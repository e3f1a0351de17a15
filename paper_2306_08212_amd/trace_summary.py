"""Summarise a rocprofv3 kernel trace of `bench.py` as markdown.

    python -m paper_2306_08212_amd.trace_summary <rocprofv3 output dir> \
        --steps K --profiled P [--kernel gemm_f64_kernel]

Three tables from the `*kernel_trace.csv` that `rocprofv3 --kernel-trace -f
csv` writes:
* the whole run, per kernel (what `--stats` reports);
* the timed moves: the K moves issued just before the profiled pass, per move
  (kernel time summed over streams, launches, average duration) and the wall
  time per move from the first to the last dispatch of the window;
* the profiled pass: the launches between the first and the last gate kernel
  (`prof_gate_kernel`, which only that pass launches), whose durations the
  HIP events of `bench.py` also measure; the average of `--kernel` there is
  the figure to set against the roofline's `avg_launch_us`.
The move boundaries come from the FP32 chain GEMMs: the profiled pass holds
P moves, which gives their number per move.
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import sys


def _name(row):
    """The kernel's bare name (the trace holds it truncated with -T, or
    demangled in full)."""
    n = row.get("Kernel_Name") or ""
    for pre in ("void ", "ctm::(anonymous namespace)::", "ctm::"):
        n = n.replace(pre, "")
    return n.split("(")[0].split("<")[0].strip()


def load(d):
    """(start, end, kernel name, stream) per dispatch, by start time; the
    stream is the trace's Stream_Id, else its Queue_Id, else 0."""
    paths = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not paths:
        raise SystemExit(f"no kernel_trace.csv under {d}")
    ev = []
    with open(paths[0]) as f:
        for r in csv.DictReader(f):
            sid = r.get("Stream_Id") or r.get("Queue_Id") or "0"
            ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _name(r), sid))
    ev.sort()
    return ev


def busy_ms(ev):
    """Time in ms during which at least one of the dispatches runs."""
    tot, cur_s, cur_e = 0, None, None
    for s, e, *_ in ev:
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot / 1e6


def table(ev, div=1.0, top=25):
    tot = collections.defaultdict(lambda: [0, 0.0])
    for s, e, n, _ in ev:
        tot[n][0] += 1
        tot[n][1] += (e - s) / 1e6
    allms = sum(v[1] for v in tot.values()) or 1.0
    out = []
    for n, (c, ms) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"| {n} | {c / div:.0f} | {ms / div:.2f} | {1e3 * ms / c:.2f} | {100 * ms / allms:.1f} |")
    return out, tot


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("dir")
    ap.add_argument("--steps", type=int, required=True, help="timed moves of the bench run")
    ap.add_argument("--profiled", type=int, default=4, help="moves of the profiled pass")
    ap.add_argument("--kernel", default="gemm_f64_kernel",
                    help="kernel (or kernels joined by +) whose average is reported")
    a = ap.parse_args(argv)
    ev = load(a.dir)
    hdr = "| kernel | launches | total ms | avg us | % |\n|---|---:|---:|---:|---:|"
    rows, _ = table(ev)
    print("### Whole run\n\n" + hdr)
    print("\n".join(rows))

    gates = [i for i, x in enumerate(ev) if x[2] == "prof_gate_kernel"]
    if not gates:
        print("\n(no gate kernels: the run has no profiled pass)")
        return 0
    g0, g1 = ev[gates[0]][0], ev[gates[-1]][1]
    prof = [x for x in ev if g0 <= x[0] <= g1 and x[2] != "prof_gate_kernel"]
    f32_prof = sum(1 for x in prof if x[2] == "gemm_f32_kernel")
    per_move = f32_prof // max(a.profiled, 1)

    before = [x for x in ev if x[0] < g0]
    f32_idx = [i for i, x in enumerate(before) if x[2] == "gemm_f32_kernel"]
    need = per_move * a.steps
    if per_move > 0 and len(f32_idx) >= need:
        # the window opens at the first chain GEMM of the first timed move;
        # the kernels of a move that precede its first chain GEMM (the
        # isometries) are counted with the move before, which evens out over
        # the window except at its ends
        i0 = f32_idx[-need]
        win = before[i0:]
        wall = (win[-1][1] - win[0][0]) / 1e6
        rows, tot = table(win, div=a.steps)
        ksum = sum(v[1] for v in tot.values()) / a.steps
        print(f"\n### Timed moves ({a.steps} moves before the profiled pass, {per_move} FP32 chain "
              f"GEMMs per move)\n")
        print(f"Wall time per move {wall / a.steps:.1f} ms; kernel time summed over streams "
              f"{ksum:.1f} ms per move; {len(win) / a.steps:.0f} launches per move.\n")
        print("| kernel | launches per move | ms per move | avg us | % |\n|---|---:|---:|---:|---:|")
        print("\n".join(rows))
        # how much of the window the GPU and each stream spend running kernels
        streams = collections.defaultdict(list)
        for x in win:
            streams[x[3]].append(x)
        print(f"\nAt least one kernel running: {busy_ms(win) / a.steps:.1f} ms of the "
              f"{wall / a.steps:.1f} ms per move.\n")
        print("| stream | launches per move | busy ms per move | % of the window |\n|---|---:|---:|---:|")
        for sid, xs in sorted(streams.items(), key=lambda kv: -len(kv[1])):
            b = busy_ms(xs)
            print(f"| {sid} | {len(xs) / a.steps:.0f} | {b / a.steps:.1f} | {100 * b / wall:.0f} |")

    rows, tot = table(prof, div=max(a.profiled, 1))
    print(f"\n### Profiled pass ({a.profiled} moves, gate kernels excluded)\n")
    print("| kernel | launches per move | ms per move | avg us | % |\n|---|---:|---:|---:|---:|")
    print("\n".join(rows))
    names = [k for k in a.kernel.split("+") if k in tot]
    if names:
        c = sum(tot[k][0] for k in names)
        ms = sum(tot[k][1] for k in names)
        print(f"\n`{a.kernel}` in the profiled pass: {c} launches, average {1e3 * ms / c:.2f} us.")
    return 0


if __name__ == "__main__":
    sys.exit(main())
