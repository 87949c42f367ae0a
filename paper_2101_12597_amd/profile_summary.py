"""Text summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2101_12597_amd.profile_summary trace <dir>/kt_kernel_stats.csv [top]
      kernel name, calls, total and average duration (microseconds), share of GPU time
  python -m paper_2101_12597_amd.profile_summary pmc <dir>/p_counter_collection.csv [top]
      per kernel: dispatches and the mean counter value per dispatch (KiB for
      FETCH_SIZE / WRITE_SIZE)
  python -m paper_2101_12597_amd.profile_summary db <dir>/<name>_results.db [top]
      the same as "trace" for a rocpd SQLite database
  python -m paper_2101_12597_amd.profile_summary mfma <dir>/p_counter_collection.csv [top]
      per kernel, from a --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE run: dispatches,
      mean duration and MFMA utilization = busy cycles summed over the SIMDs / (GPU
      cycles x SIMDs).  GRBM_GUI_ACTIVE comes summed over the XCDs, so the GPU cycles of
      a dispatch are GRBM_GUI_ACTIVE / XCDS and the SIMDs number XCDS x SIMDS_PER_XCD.
"""
import collections
import csv
import sqlite3
import sys


def trace_csv(path, top=30):
    rows = list(csv.DictReader(open(path)))
    print(f"{'kernel':<100} {'calls':>6} {'total_us':>12} {'avg_us':>11} {'pct':>6}")
    for r in rows[:top]:
        print(f"{r['Name'][:100]:<100} {int(r['Calls']):>6} {float(r['TotalDurationNs']) / 1e3:>12.1f} "
              f"{float(r['AverageNs']) / 1e3:>11.2f} {float(r['Percentage']):>6.2f}")


def pmc_csv(path, top=30):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    items = sorted(agg.items(), key=lambda kv: -sum(kv[1]))
    print(f"{'kernel':<100} {'counter':<12} {'dispatches':>10} {'mean_per_dispatch':>18}")
    for (name, counter), vals in items[:top]:
        print(f"{name[:100]:<100} {counter:<12} {len(vals):>10} {sum(vals) / len(vals):>18.1f}")


XCDS = 8
SIMDS_PER_XCD = 128  # 32 CUs x 4 SIMDs


def mfma_csv(path, top=30):
    per = collections.defaultdict(dict)
    meta = {}
    for r in csv.DictReader(open(path)):
        k = int(r["Dispatch_Id"])
        per[k][r["Counter_Name"]] = float(r["Counter_Value"])
        meta[k] = (r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0, 0])
    for k, c in per.items():
        name, dur = meta[k]
        a = agg[name]
        a[0] += 1
        a[1] += c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        a[2] += c.get("GRBM_GUI_ACTIVE", 0.0)
        a[3] += dur
    print(f"{'kernel':<100} {'dispatches':>10} {'avg_us':>10} {'mfma_util_pct':>14}")
    for name, (n, busy, gui, dur) in sorted(agg.items(), key=lambda kv: -kv[1][3])[:top]:
        util = 100.0 * busy / (gui / XCDS * XCDS * SIMDS_PER_XCD) if gui > 0 else 0.0
        print(f"{name[:100]:<100} {n:>10} {dur / n / 1e3:>10.1f} {util:>14.1f}")


def trace_db(path, top=30):
    cur = sqlite3.connect(path).cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage "
                            "from top_kernels order by total_duration desc"))
    print(f"{'kernel':<100} {'calls':>6} {'total_us':>12} {'avg_us':>11} {'pct':>6}")
    for name, calls, tot, avg, pct in rows[:top]:
        print(f"{name[:100]:<100} {calls:>6} {tot:>12.1f} {avg:>11.2f} {pct:>6.2f}")


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    top = int(sys.argv[3]) if len(sys.argv) > 3 else 30
    {"trace": trace_csv, "pmc": pmc_csv, "db": trace_db, "mfma": mfma_csv}[mode](path, top)
