"""Helpers for reading rocprofv3 output of this library's kernels.

``python -m paper_0911_4114_amd.profiling trace <results.db|kernel_trace.csv> [top]`` prints a
per-kernel Markdown table (calls, total and average duration).
``python -m paper_0911_4114_amd.profiling streams <kernel_trace.csv> <kernel>`` prints, for one
kernel (short name), its calls and average duration per HIP stream.
``python -m paper_0911_4114_amd.profiling pmc <counter_collection.csv> <kernel substring> <counter>``
prints the mean of a counter over the dispatches of the matching kernels.
``python -m paper_0911_4114_amd.profiling traffic --kernel NAME --fetch CSV --write CSV
--copy-fetch CSV --copy-write CSV --copy-bytes B --source FILE`` prints the HBM-traffic summary
of one kernel (its largest launches): FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what
the same counter reads for a plain device copy of B bytes, plus the SHA-256 of the kernel's source
file, so that a reader can tell whether the figures still describe the code. With ``--family`` the
kernel name is a prefix and the figures are the mean over every dispatch of every matching kernel
(a stage launched once per tree level, at several grid sizes)."""
import argparse
import csv
import collections
import hashlib
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


def stream_rows(path, kernel):
    """(stream id, calls, average_us) of the kernel whose short name equals ``kernel``."""
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if short_name(r["Kernel_Name"]) == kernel:
            agg[int(r["Stream_Id"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return [(sid, len(v), sum(v) / len(v)) for sid, v in sorted(agg.items())]


def pmc_mean(path, kernel, counter):
    """Mean of a PMC counter (rocprofv3 --pmc CSV) over dispatches whose name contains kernel."""
    vals = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    return sum(vals.values()) / max(len(vals), 1), len(vals)


def counter_per_dispatch(path, counter, kernel=None, largest=True, family=False):
    """Mean counter value (summed over its instances) per dispatch of the kernel whose short name
    equals ``kernel`` (any kernel if None; with ``family``, every kernel whose short name starts
    with it), over the dispatches with the largest grid (over all of them if not ``largest``)."""
    vals, grid = collections.defaultdict(float), {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = short_name(r["Kernel_Name"])
        if kernel is not None and not (name.startswith(kernel) if family else name == kernel):
            continue
        vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
        grid[r["Dispatch_Id"]] = int(r["Grid_Size"])
    if not vals:
        raise SystemExit("no %s rows for %s in %s" % (counter, kernel, path))
    g = max(grid.values()) if largest else None
    sel = [v for d, v in vals.items() if not largest or grid[d] == g]
    return sum(sel) / len(sel), len(sel), g


def file_sha256(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def traffic_summary(a):
    cf, _, _ = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw, _, _ = counter_per_dispatch(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    f, nf, gf = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel, not a.family, a.family)
    w, nw, gw = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel, not a.family, a.family)
    fs, ws = a.copy_bytes / (cf * 1024.0), a.copy_bytes / (cw * 1024.0)
    lines = [
        "kernel: %s" % (a.kernel + "*" if a.family else a.kernel),
        "grid_size: %s" % ("all" if a.family else "%d" % gf),
        "source: %s" % a.source,
        "source_sha256: %s" % file_sha256(a.source),
        "fetch_kib_per_dispatch: %.1f (%d dispatches)" % (f, nf),
        "write_kib_per_dispatch: %.1f (%d dispatches)" % (w, nw),
        "copy_bytes: %d" % a.copy_bytes,
        "copy_fetch_kib: %.1f" % cf,
        "copy_write_kib: %.1f" % cw,
        "fetch_scale: %.4f" % fs,
        "write_scale: %.4f" % ws,
        "hbm_bytes_per_dispatch: %.0f" % (1024.0 * (f * fs + w * ws)),
    ]
    return "\n".join(lines)


def traffic_total(a):
    """HBM bytes per call of a kernel group: FETCH_SIZE and WRITE_SIZE (each scaled by the copy
    probe) summed over every dispatch whose short name starts with one of the prefixes, divided
    by the number of dispatches of the kernel that runs once per call (``--per``)."""
    cf, _, _ = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw, _, _ = counter_per_dispatch(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    fs, ws = a.copy_bytes / (cf * 1024.0), a.copy_bytes / (cw * 1024.0)
    total, calls = 0.0, set()
    for path, counter, scale in ((a.fetch, "FETCH_SIZE", fs), (a.write, "WRITE_SIZE", ws)):
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = short_name(r["Kernel_Name"])
            if name == a.per:
                calls.add((path, r["Dispatch_Id"]))
            if any(name.startswith(k) for k in a.prefix):
                total += 1024.0 * scale * float(r["Counter_Value"])
    n = len(calls) // 2
    if n == 0:
        raise SystemExit("no dispatches of %s" % a.per)
    return "calls: %d\nhbm_bytes_per_call: %.0f" % (n, total / n)


def read_traffic(path):
    """key -> value (first token) of a summary written by ``traffic``."""
    out = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip().split(" (")[0]
    return out


def main(path, top=25):
    rows = trace_rows(path, top)
    print("| kernel | calls | total (us) | average (us) | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:
        print("| %s | %d | %.1f | %.1f | %.1f |" % (name, calls, tot, avg, pct))


if __name__ == "__main__":
    if sys.argv[1] == "traffic":
        ap = argparse.ArgumentParser(prog="profiling traffic")
        ap.add_argument("--kernel", required=True)
        ap.add_argument("--fetch", required=True)
        ap.add_argument("--write", required=True)
        ap.add_argument("--copy-fetch", required=True)
        ap.add_argument("--copy-write", required=True)
        ap.add_argument("--copy-bytes", type=int, required=True)
        ap.add_argument("--copy-kernel", default="__amd_rocclr_copyBuffer",
                        help="short name of the copy kernel (a device-to-device tensor copy)")
        ap.add_argument("--source", required=True)
        ap.add_argument("--family", action="store_true",
                        help="--kernel is a name prefix; average over all matching dispatches")
        print(traffic_summary(ap.parse_args(sys.argv[2:])))
    elif sys.argv[1] == "traffic-total":
        ap = argparse.ArgumentParser(prog="profiling traffic-total")
        ap.add_argument("--prefix", action="append", required=True,
                        help="short-name prefix of the group's kernels (repeatable)")
        ap.add_argument("--per", required=True, help="short name of a kernel run once per call")
        ap.add_argument("--fetch", required=True)
        ap.add_argument("--write", required=True)
        ap.add_argument("--copy-fetch", required=True)
        ap.add_argument("--copy-write", required=True)
        ap.add_argument("--copy-bytes", type=int, required=True)
        ap.add_argument("--copy-kernel", default="__amd_rocclr_copyBuffer")
        print(traffic_total(ap.parse_args(sys.argv[2:])))
    elif sys.argv[1] == "trace":
        main(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25)
    elif sys.argv[1] == "streams":
        print("| stream | calls | average (us) |")
        print("|---|---|---|")
        for sid, calls, avg in stream_rows(sys.argv[2], sys.argv[3]):
            print("| %d | %d | %.1f |" % (sid, calls, avg))
    elif sys.argv[1] == "pmc":
        m, cnt = pmc_mean(sys.argv[2], sys.argv[3], sys.argv[4])
        print("%s %s: mean %.1f over %d dispatches" % (sys.argv[3], sys.argv[4], m, cnt))
