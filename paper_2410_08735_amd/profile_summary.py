"""Summarise a rocprofv3 kernel trace (``--kernel-trace --output-format csv``).

    python -m paper_2410_08735_amd.profile_summary <prefix>_kernel_trace.csv [top]
    python -m paper_2410_08735_amd.profile_summary <prefix>_counter_collection.csv [top]

For a kernel trace: two markdown tables, the kernels between the first two
region markers (``rte::k_region_marker``, enqueued by ``rte_prof_mark``
around a timed region) and the kernels of the whole process.  For a counter
collection (``--pmc``): the mean counter value per dispatch of each kernel
between the first and second markers and between the third and fourth (in
bench.py: the timed region and the calibration copy; in its learned leg, the
network's training and the FGMRES-MLP solves).
Kernel names are shortened to their qualified name and template arguments.
"""
import collections
import csv
import sys

MARKER = "k_region_marker"


def _short(name):
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    s = "".join(out)
    return s[5:] if s.startswith("void ") else s


def _table(rows, title, top):
    agg = collections.defaultdict(lambda: [0, 0])
    for r in rows:
        a = agg[_short(r["Kernel_Name"])]
        a[0] += 1
        a[1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    tot = sum(v[1] for v in agg.values()) or 1
    lines = [f"### {title}", "",
             f"busy {tot / 1e6:.2f} ms in {sum(v[0] for v in agg.values())} dispatches", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, (c, ns) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"| `{name}` | {c} | {ns / 1e6:.3f} | {ns / c / 1e3:.1f} | {100 * ns / tot:.1f} |")
    return "\n".join(lines) + "\n"


def summarise(path, top=25):
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    marks = [i for i, r in enumerate(rows) if MARKER in r["Kernel_Name"]]
    body = [r for r in rows if MARKER not in r["Kernel_Name"]]
    out = []
    if len(marks) >= 2:
        region = [r for r in rows[marks[0] + 1:marks[1]] if MARKER not in r["Kernel_Name"]]
        span = int(rows[marks[1]]["Start_Timestamp"]) - int(rows[marks[0]]["End_Timestamp"])
        out.append(_table(region, f"timed region (between markers, {span / 1e6:.2f} ms wall on the GPU)", top))
    out.append(_table(body, "whole process", top))
    return "\n".join(out)


def summarise_counters(path, top=25):
    """Mean counter value per dispatch, per kernel, between the timed-region
    markers and between the copy-probe markers.  A dispatch whose counter sum
    is below 0.1 % of the kernel's largest did no work (FGMRES enqueues a step
    before it knows that every instance has converged); such dispatches are
    counted in their own column and left out of the mean."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
    # one row per (dispatch, counter): a marker is the first row of its dispatch
    marks = [i for i, r in enumerate(rows) if MARKER in r["Kernel_Name"]
             and (i == 0 or rows[i - 1]["Dispatch_Id"] != r["Dispatch_Id"])]
    out = []
    for title, (a, b) in (("between markers 1 and 2", (0, 1)), ("between markers 3 and 4", (2, 3))):
        if len(marks) <= b:
            continue
        per = collections.defaultdict(lambda: collections.defaultdict(dict))  # kernel -> dispatch -> counter
        for r in rows[marks[a] + 1:marks[b]]:
            if MARKER in r["Kernel_Name"]:
                continue
            k = _short(r["Kernel_Name"])
            d = per[k][r["Dispatch_Id"]]
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        names = sorted({c for v in per.values() for d in v.values() for c in d})
        out += [f"### {title}", "", "| kernel | dispatches with work | no-work dispatches | "
                + " | ".join(f"mean {c} per dispatch" for c in names) + " |",
                "|---|---:|---:|" + "---:|" * len(names)]
        tot = {k: sum(sum(d.values()) for d in v.values()) for k, v in per.items()}
        for k in sorted(per, key=lambda k: -tot[k])[:top]:
            big = max(sum(d.values()) for d in per[k].values())
            work = [d for d in per[k].values() if sum(d.values()) >= 1e-3 * big]
            vals = [sum(d.get(c, 0.0) for d in work) / len(work) for c in names]
            out.append(f"| `{k}` | {len(work)} | {len(per[k]) - len(work)} | "
                       + " | ".join(f"{v:.1f}" for v in vals) + " |")
        out.append("")
    return "\n".join(out)


if __name__ == "__main__":
    top = int(sys.argv[2]) if len(sys.argv) > 2 else 25
    if sys.argv[1].endswith("counter_collection.csv"):
        print(summarise_counters(sys.argv[1], top))
    else:
        print(summarise(sys.argv[1], top))
