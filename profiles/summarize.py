"""Print a per-kernel summary (calls, total and average duration) from a rocprofv3 results
database (SQLite, --kernel-trace) as a Markdown table."""
import sqlite3
import sys


def main(db_path, top=25):
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels limit ?", (top,)).fetchall()
    print("| kernel | calls | total (us) | average (us) | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:
        short = name.replace("(anonymous namespace)::", "").replace("void ", "")
        short = short.replace("ffmm::", "").split("(")[0]
        print("| %s | %d | %.1f | %.1f | %.1f |" % (short, calls, tot / 1e3 if tot > 1e6 else tot,
                                                   avg, pct))


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 25)
