"""Per-kernel summary (calls, average/min/max duration, grid, registers, LDS) of a
rocprofv3 --kernel-trace run, from its CSV trace or its SQLite database:

    python -m paper_1609_04104_amd.prof_summary RUN_kernel_trace.csv
    python -m paper_1609_04104_amd.prof_summary RUN_results.db
"""
import csv
import sqlite3
import sys
from collections import defaultdict


def _rows_csv(path):
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            yield (r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                   int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]), int(r["Workgroup_Size_X"]),
                   int(r["VGPR_Count"]) + int(r["Accum_VGPR_Count"]), int(r["LDS_Block_Size"]),
                   int(r["Scratch_Size"]))


def _rows_db(path):
    db = sqlite3.connect(path)
    for name, dur, gx, gy, wx in db.execute(
            "select name, end - start, grid_x, grid_y, workgroup_x from kernels"):
        yield name, dur, gx, gy, wx, -1, -1, -1


def summarize(path, out=sys.stdout):
    rows = _rows_csv(path) if path.endswith(".csv") else _rows_db(path)
    acc = defaultdict(list)
    meta = {}
    for name, dur, gx, gy, wx, vgpr, lds, scratch in rows:
        key = (name, gx, gy)
        acc[key].append(dur)
        meta[key] = (wx, vgpr, lds, scratch)
    order = sorted(acc, key=lambda k: -sum(acc[k]))
    print("| kernel | calls | avg us | min us | max us | total us | grid (work-items) | block | VGPR | LDS B | scratch B |",
          file=out)
    print("|---|---|---|---|---|---|---|---|---|---|---|", file=out)
    for key in order:
        d = acc[key]
        name, gx, gy = key
        wx, vgpr, lds, scratch = meta[key]
        short = name.replace("tsl::(anonymous namespace)::", "").replace("tsl::", "").split("(")[0]
        if len(short) > 70:
            short = short[:67] + "..."
        print(f"| {short} | {len(d)} | {sum(d) / len(d) / 1e3:.2f} | {min(d) / 1e3:.2f} | {max(d) / 1e3:.2f} | "
              f"{sum(d) / 1e3:.1f} | {gx} x {gy} | {wx} | {vgpr} | {lds} | {scratch} |", file=out)


if __name__ == "__main__":
    summarize(sys.argv[1])
