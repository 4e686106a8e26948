"""Condense a rocprofv3 kernel trace (``<prefix>_kernel_trace.csv``) into a short table:
one line per kernel and launch grid (so the workloads of one run stay apart), with the
number of dispatches, mean / min / max duration, VGPRs and LDS bytes per workgroup.

    python -m paper_2606_15622_amd.prof_summary TRACE.csv [--title T] [--command C]
"""
import argparse
import csv
import re
from collections import defaultdict


def short(name):
    name = re.sub(r"^void ", "", name)
    name = re.sub(r"\(.*$", "", name)
    return name.replace("fpg::", "")


def summarize(path, title="", command=""):
    groups = defaultdict(list)
    meta = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            k = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
            groups[k].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            meta[k] = (r.get("VGPR_Count", ""), r.get("Accum_VGPR_Count", ""), r.get("LDS_Block_Size", ""),
                       r.get("Workgroup_Size_X", ""))
    out = []
    if title:
        out.append(f"# {title}")
    if command:
        out.append(f"# command: {command}")
    out.append("# from rocprofv3 --kernel-trace; durations in microseconds; grid = work-items")
    out.append(f"{'kernel':<46} {'grid':>10} {'wg':>4} {'calls':>6} {'mean_us':>9} {'min_us':>9} "
               f"{'max_us':>9} {'vgpr':>5} {'agpr':>5} {'lds':>6}")
    total = sum(sum(v) for v in groups.values())
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    for (name, grid), d in rows:
        vg, ag, lds, wg = meta[(name, grid)]
        out.append(f"{name[:46]:<46} {grid:>10} {wg:>4} {len(d):>6} {sum(d) / len(d) / 1e3:>9.2f} "
                   f"{min(d) / 1e3:>9.2f} {max(d) / 1e3:>9.2f} {vg:>5} {ag:>5} {lds:>6}")
    out.append(f"# total kernel time {total / 1e6:.3f} ms over {sum(len(v) for v in groups.values())} dispatches")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    print(summarize(a.trace, a.title, a.command))


if __name__ == "__main__":
    main()
