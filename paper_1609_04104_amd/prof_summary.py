"""Prints a per-kernel summary (calls, average and total duration) of a
rocprofv3 --kernel-trace database:  python -m paper_1609_04104_amd.prof_summary RUN_results.db"""
import sqlite3
import sys


def main(path):
    db = sqlite3.connect(path)
    rows = db.execute(
        "select name, count(*), avg(end - start) / 1000.0, sum(end - start) / 1000.0, grid_x, grid_y, "
        "workgroup_x from kernels group by name, grid_x, grid_y order by sum(end - start) desc").fetchall()
    print("| kernel | calls | avg us | total us | grid (work-items) | block |")
    print("|---|---|---|---|---|---|")
    for name, n, avg, tot, gx, gy, wx in rows:
        short = name.replace("tsl::(anonymous namespace)::", "").split("(")[0]
        print(f"| {short} | {n} | {avg:.2f} | {tot:.1f} | {gx} x {gy} | {wx} |")


if __name__ == "__main__":
    main(sys.argv[1])
