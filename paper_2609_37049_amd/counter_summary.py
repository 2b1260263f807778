"""HBM traffic of the solver's stencil launches from two rocprofv3 counter runs.

    python -m paper_2609_37049_amd.counter_summary FETCH.csv WRITE.csv --grid G --key KEY
           [--tile Y,T] [--note TEXT] [--update profiles/stencil_traffic.json]

FETCH.csv and WRITE.csv are the counter_collection.csv files of
`rocprofv3 --pmc FETCH_SIZE` and `rocprofv3 --pmc WRITE_SIZE` runs of
paper_2609_37049_amd/profile_stencil.py.  The counters are in KiB per
dispatch; the harness's last kernels copy 256 MiB, and the ratio of the bytes
that copy moved to what the counters report for it calibrates each counter.
The launches counted are the even-odd BF16 stencil instances of the full
operator (buffer loads, LDS staging, no mask) with grid G (the solver's block
width), in the solver's own mix of launches.  Prints a markdown table and,
with --update, writes the calibrated bytes per launch under KEY, with the hash
of the stencil sources they were taken on.
"""
import argparse
import csv
import json
import os
import sys
from collections import defaultdict

COPY_BYTES = 256 << 20


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _kib_by_dispatch(path):
    out = {}
    for r in _rows(path):
        out[int(r["Dispatch_Id"])] = (r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]))
    return out


def _copy_factor(disp):
    """Bytes per counted KiB for the 256 MiB device copy (the last dispatches)."""
    ids = sorted(disp)
    last = [disp[i] for i in ids[-3:]]
    vals = [v for name, grid, v in last if "copy" in name.lower() or "elementwise" in name.lower()]
    if not vals:
        sys.exit("no copy kernel among the last dispatches")
    kib = sum(vals) / len(vals)
    return COPY_BYTES / (kib * 1024.0), kib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch")
    ap.add_argument("write")
    ap.add_argument("--grid", type=int, required=True)
    ap.add_argument("--key", required=True)
    ap.add_argument("--tile", default="")
    ap.add_argument("--note", default="")
    ap.add_argument("--update", default="")
    args = ap.parse_args()
    fe, wr = _kib_by_dispatch(args.fetch), _kib_by_dispatch(args.write)
    ff, fk = _copy_factor(fe)
    wf, wk = _copy_factor(wr)
    per = defaultdict(lambda: [0, 0.0, 0.0])
    for i, (name, grid, v) in fe.items():
        inst = name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0].strip()
        if grid != args.grid or not inst.startswith("k_dslash<IOBF") or not inst.endswith("true, true, true, false>"):
            continue
        w = wr.get(i)
        if w is None:
            continue
        per[inst][0] += 1
        per[inst][1] += v * 1024.0 * ff
        per[inst][2] += w[2] * 1024.0 * wf
    n = sum(c for c, _, _ in per.values())
    if not n:
        sys.exit("no matching stencil dispatches")
    rd = sum(r for _, r, _ in per.values()) / n
    wt = sum(w for _, _, w in per.values()) / n
    print("Calibration: the copy reads FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB, factors %.3f (fetch) "
          "and %.3f (write)." % (fk, wk, ff, wf))
    print()
    print("| launch | count | calibrated read MB | calibrated write MB |")
    print("|---|---|---|---|")
    for inst, (c, r, w) in sorted(per.items()):
        print("| `%s` | %d | %.1f | %.1f |" % (inst, c, r / c / 1e6, w / c / 1e6))
    print()
    print("Solver mix: %.1f MB of HBM traffic per launch (%.1f read, %.1f write) over %d launches."
          % ((rd + wt) / 1e6, rd / 1e6, wt / 1e6, n))
    if args.update:
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        sys.path.insert(0, root)
        import bench
        d = json.load(open(args.update)) if os.path.exists(args.update) else {}
        d[args.key] = {"source_hash": bench.stencil_hash(), "bytes_per_launch": round(rd + wt),
                       "read_bytes": round(rd), "write_bytes": round(wt), "fetch_factor": round(ff, 3),
                       "write_factor": round(wf, 3), "tile": args.tile, "note": args.note}
        with open(args.update, "w") as f:
            json.dump(d, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
