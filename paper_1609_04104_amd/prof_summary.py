"""Summaries of rocprofv3 runs.

Per-kernel durations (calls, average/min/max, grid, registers, LDS) of a
--kernel-trace run, from its CSV trace or its SQLite database:

    python -m paper_1609_04104_amd.prof_summary RUN_kernel_trace.csv
    python -m paper_1609_04104_amd.prof_summary RUN_results.db

Per-dispatch HBM bytes of every kernel from two --pmc runs (FETCH_SIZE, then
WRITE_SIZE) of a program that first makes one plain device copy of a known
size (bench.py --copy-calib-mib M), written as a JSON record keyed by kernel:

    python -m paper_1609_04104_amd.prof_summary counters FETCH_counter_collection.csv \
        WRITE_counter_collection.csv M OUT.json
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




# ----------------------------------------------------------------------------- byte counters
def source_sha():
    """SHA-256 over the HIP sources of the library (names and contents, sorted),
    so a counter record can tell whether the kernels changed since it was taken."""
    import glob
    import hashlib
    import os
    h = hashlib.sha256()
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for p in sorted(glob.glob(os.path.join(here, "*.hip")) + glob.glob(os.path.join(here, "*.hpp"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _per_dispatch(path, counter):
    acc, disp, grid = defaultdict(float), defaultdict(set), {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = r["Kernel_Name"].replace("tsl::(anonymous namespace)::", "").replace("tsl::", "").split("(")[0]
            key = f"{key} [grid {r['Grid_Size']}]"
            acc[key] += float(r["Counter_Value"])
            disp[key].add(r["Dispatch_Id"])
            grid[key] = int(r["Grid_Size"])
    return {k: acc[k] / len(disp[k]) for k in acc}, {k: len(disp[k]) for k in acc}, grid


def counters(fetch_csv, write_csv, copy_mib, out):
    """Per-dispatch HBM bytes of every kernel from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter
    reads for the reference copy of copy_mib MiB (the copyBuffer dispatch of
    that size) so that the figures are true bytes."""
    import json
    fetch, nf, grid = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write, _, _ = _per_dispatch(write_csv, "WRITE_SIZE")
    kib = copy_mib * 1024.0
    ref = [k for k in write if "copyBuffer" in k and abs(write[k] - kib) < 0.02 * kib]
    if not ref:
        raise SystemExit("no reference copy dispatch of the given size in the WRITE_SIZE run")
    fscale = kib / fetch[ref[0]]
    wscale = kib / write[ref[0]]
    rec = {"source_sha": source_sha(), "reference_copy_mib": copy_mib,
           "fetch_scale": fscale, "write_scale": wscale, "kernels": {}}
    for k in sorted(fetch):
        if k not in write:
            continue
        rec["kernels"][k] = {"fetch_bytes": fetch[k] * 1024.0 * fscale, "write_bytes": write[k] * 1024.0 * wscale,
                             "dispatches": nf[k], "grid": grid[k]}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(f"fetch scale {fscale:.3f}, write scale {wscale:.3f}, {len(rec['kernels'])} kernels -> {out}")
    print("\n| kernel | dispatches | read MiB | written MiB |\n|---|---|---|---|")
    for k, v in rec["kernels"].items():
        if k.startswith("void k_"):
            print(f"| {k} | {v['dispatches']} | {v['fetch_bytes'] / 2**20:.1f} | {v['write_bytes'] / 2**20:.1f} |")


if __name__ == "__main__":
    if sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5])
    else:
        summarize(sys.argv[1])
