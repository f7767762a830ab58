"""Helpers for reading rocprofv3 output of this library's kernels.

``python -m paper_0911_4114_amd.profiling trace <results.db|kernel_trace.csv> [top]`` prints a
per-kernel Markdown table (calls, total and average duration).
``python -m paper_0911_4114_amd.profiling pmc <counter_collection.csv> <kernel substring> <counter>``
prints the mean of a counter over the dispatches of the matching kernels."""
import csv
import collections
import sqlite3
import sys


def short_name(name):
    n = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("ffmm::", "")
    n = n.split("(")[0]
    return n.replace("HIP_vector_type<float, 2u>", "float2").replace("HIP_vector_type<double, 2u>",
                                                                     "double2")


def trace_rows(path, top=25):
    """(name, calls, total_us, average_us, percent) per kernel, largest total first."""
    if path.endswith(".db"):
        cur = sqlite3.connect(path).cursor()
        rows = cur.execute("select name, total_calls, total_duration, average, percentage "
                           "from top_kernels limit ?", (top,)).fetchall()
        return [(short_name(a), b, c, d, e) for a, b, c, d, e in rows]
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[short_name(r["Kernel_Name"])].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in agg.values())
    rows = [(k, len(v), sum(v), sum(v) / len(v), 100.0 * sum(v) / total) for k, v in agg.items()]
    rows.sort(key=lambda r: -r[2])
    return rows[:top]


def pmc_mean(path, kernel, counter):
    """Mean of a PMC counter (rocprofv3 --pmc CSV) over dispatches whose name contains kernel."""
    vals = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    return sum(vals.values()) / max(len(vals), 1), len(vals)


def main(path, top=25):
    rows = trace_rows(path, top)
    print("| kernel | calls | total (us) | average (us) | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:
        print("| %s | %d | %.1f | %.1f | %.1f |" % (name, calls, tot, avg, pct))


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        main(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25)
    elif sys.argv[1] == "pmc":
        m, cnt = pmc_mean(sys.argv[2], sys.argv[3], sys.argv[4])
        print("%s %s: mean %.1f over %d dispatches" % (sys.argv[3], sys.argv[4], m, cnt))
