"""Summarize a rocprofv3 kernel-trace database (``*_results.db``) as text:
kernel name, calls, total and average duration, share of GPU time."""
import sqlite3
import sys


def main(db, top=30):
    cur = sqlite3.connect(db).cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage "
                            "from top_kernels order by total_duration desc"))
    print(f"{'kernel':<100} {'calls':>6} {'total_us':>11} {'avg_us':>10} {'pct':>6}")
    for name, calls, tot, avg, pct in rows[:top]:
        print(f"{name[:100]:<100} {calls:>6} {tot:>11.1f} {avg:>10.2f} {pct:>6.2f}")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 30)
