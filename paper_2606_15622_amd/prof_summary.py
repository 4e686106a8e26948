"""Short text summaries of rocprofv3 output, for the profiles/ directory.

    python -m paper_2606_15622_amd.prof_summary trace TRACE.csv [--title T] [--command C]
        one line per kernel and launch grid of a --kernel-trace run: dispatches, mean /
        min / max duration, VGPRs, LDS bytes per workgroup
    python -m paper_2606_15622_amd.prof_summary copy
        a plain device copy of 256 MiB (three times), the known-size reference for the
        FETCH_SIZE / WRITE_SIZE counters
    python -m paper_2606_15622_amd.prof_summary alu SQ.csv [SQ2.csv ...] --match REGEX@GRID [...]
            --source FILE
        VALU-busy cycles of an entry point (SQ_ACTIVE_INST_VALU), for the ALU roofline
    python -m paper_2606_15622_amd.prof_summary counters --fetch F.csv --write W.csv
            --copy-fetch CF.csv --copy-write CW.csv --match REGEX@GRID [--match ...]
            --source FILE [--source FILE ...] [--title T] [--command C]
        HBM bytes per launch of an entry point: the kernels matching each REGEX at its
        grid, summed, each counter scaled by bytes / counter of the reference copy; the
        listed sources are hashed so that a reader can tell whether a kernel changed since
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


COPY_BYTES = 256 * 1024 * 1024


def copy_reference():
    import torch
    a = torch.ones(COPY_BYTES // 4, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied", COPY_BYTES >> 20, "MiB x 3")


def _counter(path, name, kernel_re=None, grid=None):
    """Per-dispatch values (KiB) of one counter, grouped by dispatch id."""
    vals = defaultdict(float)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != name:
                continue
            if kernel_re and not re.search(kernel_re, r["Kernel_Name"]):
                continue
            if grid is not None and int(r["Grid_Size"]) != grid:
                continue
            vals[(r["Kernel_Name"], r["Dispatch_Id"])] += float(r["Counter_Value"])
    return vals


def counters(a):
    import hashlib
    cf = _counter(a.copy_fetch, "FETCH_SIZE")
    cw = _counter(a.copy_write, "WRITE_SIZE")
    # the copy is the dispatch with the largest values
    ref_f = max(cf.values()) * 1024.0
    ref_w = max(cw.values()) * 1024.0
    kf = COPY_BYTES / ref_f
    kw = COPY_BYTES / ref_w
    out = []
    if a.title:
        out.append(f"# {a.title}")
    if a.command:
        out.append(f"# command: {a.command}")
    out.append("# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (separate runs), KiB per dispatch;")
    out.append("# scaled by the bytes a plain 256 MiB device copy moves per counted byte")
    out.append(f"copy_factor_fetch: {kf:.4f}")
    out.append(f"copy_factor_write: {kw:.4f}")
    tot = 0.0
    pats = [(m.rsplit("@", 1)[0], int(m.rsplit("@", 1)[1])) for m in a.match]

    def window(path, name):
        # dispatches of one workload lie between the first dispatch of the first pattern
        # and the last dispatch of the last one (other workloads may run the same kernels
        # at the same grid, e.g. a grid-stride kernel)
        lo = min(int(k[1]) for k in _counter(path, name, *pats[0]))
        hi = max(int(k[1]) for k in _counter(path, name, *pats[-1]))
        return lo, hi

    fwin, wwin = window(a.fetch, "FETCH_SIZE"), window(a.write, "WRITE_SIZE")
    for kre, grid in pats:
        fd = {k: v for k, v in _counter(a.fetch, "FETCH_SIZE", kre, grid).items()
              if fwin[0] <= int(k[1]) <= fwin[1]}
        wd = {k: v for k, v in _counter(a.write, "WRITE_SIZE", kre, grid).items()
              if wwin[0] <= int(k[1]) <= wwin[1]}
        for name in sorted({k[0] for k in fd}):
            fv = [v for k, v in fd.items() if k[0] == name]
            wv = [v for k, v in wd.items() if k[0] == name]
            f = sum(fv) / len(fv) * 1024.0 * kf
            w = sum(wv) / len(wv) * 1024.0 * kw if wv else 0.0
            short = re.sub(r"\(.*$", "", name)
            out.append(f"kernel: {short} grid {grid} dispatches {len(fv)} fetch_bytes {f:.0f} "
                       f"write_bytes {w:.0f}")
            tot += f + w
    out.append(f"traffic_bytes_per_launch: {tot:.0f}")
    for src in a.source:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        out.append(f"source: {src} {digest}")
    return "\n".join(out)


def instruction_mix(a):
    """Per kernel and grid: waves, wave instructions per wave (VALU, LDS, SALU, vector
    memory reads and writes) from one rocprofv3 --pmc run of SQ counters, and the VALU
    time they imply at four cycles per wave instruction on 1024 SIMDs at 2.4 GHz."""
    rows = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(a.csv)):
        name = re.sub(r"\(.*$", "", re.sub(r"^void ", "", r["Kernel_Name"])).replace("fpg::", "")
        if a.match and not re.search(a.match, name):
            continue
        rows[(name, int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    avg = lambda v: sum(v) / len(v) if v else 0.0
    out = []
    if a.title:
        out.append(f"# {a.title}")
    if a.command:
        out.append(f"# command: {a.command}")
    out.append("# SQ_* counters summed over the chip per dispatch, averaged over dispatches; "
               "instructions are wave instructions")
    out.append(f"{'kernel':<40}{'grid':>9}{'waves':>8}{'valu/w':>8}{'lds/w':>7}{'salu/w':>7}"
               f"{'vmrd/w':>7}{'vmwr/w':>7}{'valu_us':>9}")
    for key in sorted(rows):
        c = rows[key]
        w = avg(c.get("SQ_WAVES", []))
        if w <= 0:
            continue
        valu = avg(c.get("SQ_INSTS_VALU", []))
        us = valu * 4.0 / (1024 * 2.4e9) * 1e6
        out.append(f"{key[0][:40]:<40}{key[1]:>9}{w:>8.0f}{valu / w:>8.0f}"
                   f"{avg(c.get('SQ_INSTS_LDS', [])) / w:>7.0f}{avg(c.get('SQ_INSTS_SALU', [])) / w:>7.0f}"
                   f"{avg(c.get('SQ_INSTS_VMEM_RD', [])) / w:>7.1f}{avg(c.get('SQ_INSTS_VMEM_WR', [])) / w:>7.1f}"
                   f"{us:>9.1f}")
    return "\n".join(out)


def alu(a):
    """VALU work of an entry point from one rocprofv3 --pmc run of SQ counters (SQ_WAVES,
    SQ_ACTIVE_INST_VALU, SQ_INSTS_VALU and the VALU classes): per kernel at its grid the
    waves, VALU instructions and VALU-busy cycles per wave (SQ_ACTIVE_INST_VALU counts
    quad-cycles), and per launch of the entry point the VALU-busy SIMD cycles summed over
    its kernels; the listed sources are hashed as for the traffic summary."""
    import hashlib
    # several passes (rocprofv3 collects a limited set of SQ counters per run): each
    # counter is averaged over the dispatches of the pass that collected it
    rows = defaultdict(lambda: defaultdict(list))
    for path in a.csv:
        for r in csv.DictReader(open(path)):
            rows[(r["Kernel_Name"], int(r["Grid_Size"]))][r["Counter_Name"]].append(
                float(r["Counter_Value"]))
    avg = lambda v: sum(v) / len(v) if v else 0.0
    out = []
    if a.title:
        out.append(f"# {a.title}")
    if a.command:
        out.append(f"# command: {a.command}")
    out.append("# SQ counters summed over the chip per dispatch, averaged over dispatches; instructions are "
               "wave instructions; busy = SQ_ACTIVE_INST_VALU x 4 (quad-cycles)")
    tot = 0.0
    for m in a.match:
        kre, grid = m.rsplit("@", 1)[0], int(m.rsplit("@", 1)[1])
        for (name, g), c in sorted(rows.items()):
            if g != grid or not re.search(kre, name):
                continue
            w = avg(c.get("SQ_WAVES", []))
            busy = avg(c.get("SQ_ACTIVE_INST_VALU", [])) * 4.0
            per = lambda k: avg(c.get(k, [])) / w if w else 0.0
            line = (f"kernel: {short(name)} grid {grid} waves {w:.0f} "
                    f"valu_per_wave {per('SQ_INSTS_VALU'):.1f} salu_per_wave {per('SQ_INSTS_SALU'):.1f} "
                    f"lds_per_wave {per('SQ_INSTS_LDS'):.1f} vmem_per_wave "
                    f"{per('SQ_INSTS_VMEM_RD') + per('SQ_INSTS_VMEM_WR'):.1f}")
            for key, cs in (("trans_f32", ["SQ_INSTS_VALU_TRANS_F32"]), ("int32", ["SQ_INSTS_VALU_INT32"]),
                            ("int64", ["SQ_INSTS_VALU_INT64"]), ("fma_f32", ["SQ_INSTS_VALU_FMA_F32"]),
                            ("f64", ["SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
                                     "SQ_INSTS_VALU_MUL_F64"])):
                if all(k in c for k in cs):
                    line += f" {key}_per_wave {sum(per(k) for k in cs):.1f}"
            out.append(line + f" busy_cycles_per_wave {busy / w if w else 0.0:.1f} busy_cycles {busy:.0f}")
            tot += busy
    out.append(f"valu_busy_cycles_per_launch: {tot:.0f}")
    for src in a.source:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        out.append(f"source: {src} {digest}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("trace")
    t.add_argument("--title", default="")
    t.add_argument("--command", default="")
    sub.add_parser("copy")
    m = sub.add_parser("mix")
    m.add_argument("csv")
    m.add_argument("--match", default="")
    m.add_argument("--title", default="")
    m.add_argument("--command", default="")
    c = sub.add_parser("counters")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write"):
        c.add_argument(k, required=True)
    c.add_argument("--match", action="append", required=True,
                   help="REGEX@GRID: kernels of one launch of the entry point (repeatable)")
    c.add_argument("--source", action="append", default=[])
    c.add_argument("--title", default="")
    c.add_argument("--command", default="")
    v = sub.add_parser("alu")
    v.add_argument("csv", nargs="+")
    v.add_argument("--match", action="append", required=True, help="REGEX@GRID (repeatable)")
    v.add_argument("--source", action="append", default=[])
    v.add_argument("--title", default="")
    v.add_argument("--command", default="")
    a = ap.parse_args()
    if a.cmd == "alu":
        print(alu(a))
        return
    if a.cmd == "trace":
        print(summarize(a.trace, a.title, a.command))
    elif a.cmd == "copy":
        copy_reference()
    elif a.cmd == "mix":
        print(instruction_mix(a))
    else:
        print(counters(a))


if __name__ == "__main__":
    main()
