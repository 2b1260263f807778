"""Summarise a rocprofv3 kernel trace of the benchmark as markdown tables.

    python -m paper_2609_37049_amd.trace_summary <dir with *_kernel_trace.csv> [--top 20] [--lanes 64]

Prints the top kernels by total time (from the trace itself) and the Wilson-
clover stencil launches grouped by instance and grid size, so that the
average duration of the benchmark's dominant launches (the unmasked even-odd
BF16 stencil at the solver's block width) can be set beside the bench's own
event-timed average.
"""
import argparse
import csv
import glob
import os
import re
import sys
from collections import defaultdict


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(names)


def _short(name):
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"\s*\[clone[^\]]*\]", "", name)
    name = name.replace("void ", "")
    return re.sub(r"\(.*\)$", "", name).strip()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--top", type=int, default=20)
    args = ap.parse_args()
    files = glob.glob(os.path.join(args.dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        sys.exit("no *kernel_trace.csv under %s" % args.dir)
    per = defaultdict(list)       # kernel -> durations (us)
    shape = defaultdict(list)     # (kernel, grid) -> durations
    for f in files:
        for r in _rows(f):
            name = _short(_col(r, "Kernel_Name"))
            dur = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
            grid = int(_col(r, "Grid_Size", "Grid_Size_X"))
            per[name].append(dur)
            shape[(name, grid)].append(dur)
    total = sum(sum(v) for v in per.values())
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---|---|---|---|")
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[: args.top]:
        print("| `%s` | %d | %.1f | %.1f | %.1f |" % (name, len(v), sum(v) / 1e3, sum(v) / len(v),
                                                      100 * sum(v) / total))
    print()
    print("| stencil instance | grid (threads) | calls | avg us |")
    print("|---|---|---|---|")
    for (name, grid), v in sorted(shape.items(), key=lambda kv: -sum(kv[1])):
        if not name.startswith("k_dslash"):
            continue
        print("| `%s` | %d | %d | %.1f |" % (name, grid, len(v), sum(v) / len(v)))


if __name__ == "__main__":
    main()
