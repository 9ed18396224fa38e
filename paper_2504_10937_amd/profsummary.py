"""Write a short markdown summary of rocprofv3 output for one kernel.

usage: python -m paper_2504_10937_amd.profsummary <kernel substring> <out.md> <command string>
       <kernel_stats.csv> [<fetch counter_collection.csv> <write counter_collection.csv>]
       python -m paper_2504_10937_amd.profsummary --top <N> <out.md> <title> <command string> <kernel_stats.csv>
       python -m paper_2504_10937_amd.profsummary --counters <kernel substring> <out.md> <command string>
       <counter_collection.csv>   (every counter of the file, averaged per dispatch of the kernel)

The FETCH_SIZE / WRITE_SIZE passes must come from runs that first launched a
device copy of known size (bench.py --copy-calib-mib); the copy's counters
give the scale factors that turn the counters into bytes.
"""
import csv
import hashlib
import os
import sys


def per_dispatch(path, kernel, counter):
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    return sum(vals) / len(vals) if vals else None


def copy_value(path, counter):
    best = None
    for r in csv.DictReader(open(path)):
        if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer") and r["Counter_Name"] == counter:
            v = float(r["Counter_Value"])
            best = v if best is None else max(best, v)
    return best


def top(n, out, title, cmd, stats):
    rows = list(csv.DictReader(open(stats)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 --kernel-trace --stats: %s" % title, "", "command: `%s`" % cmd, "",
             "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[:n]:
        name = r["Name"].replace("lds::(anonymous namespace)::", "").split("(")[0][:70]
        lines.append("| %s | %s | %.1f | %.2f | %.1f |" % (name, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                         float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(kernel, out, cmd, path):
    vals = {}
    for r in csv.DictReader(open(path)):
        if kernel in r["Kernel_Name"]:
            vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    src = open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "fw.hip"), "rb").read()
    lines = ["# rocprofv3 counters: %s" % kernel, "",
             "kernel source sha256[:16]: `%s` (paper_2504_10937_amd/csrc/fw.hip)" % hashlib.sha256(src).hexdigest()[:16],
             "", "command: `%s`" % cmd, "", "| counter | dispatches | mean per dispatch |", "|---|---|---|"]
    for name in sorted(vals):
        v = vals[name]
        lines.append("| %s | %d | %.6e |" % (name, len(v), sum(v) / len(v)))
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    if sys.argv[1] == "--top":
        return top(int(sys.argv[2]), *sys.argv[3:7])
    if sys.argv[1] == "--counters":
        return counters(*sys.argv[2:6])
    kernel, out, cmd, stats = sys.argv[1:5]
    rows = [r for r in csv.DictReader(open(stats)) if kernel in r["Name"]]
    src = open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "fw.hip"), "rb").read()
    lines = ["# rocprofv3 summary: %s" % kernel, "",
             "kernel source sha256[:16]: `%s` (paper_2504_10937_amd/csrc/fw.hip)" % hashlib.sha256(src).hexdigest()[:16],
             "", "command: `%s`" % cmd, "", "| kernel | calls | avg ns | min ns | max ns | total % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| %s | %s | %.0f | %s | %s | %.1f |" % (r["Name"][:90], r["Calls"], float(r["AverageNs"]),
                                                           r["MinNs"], r["MaxNs"], float(r["Percentage"])))
    if len(sys.argv) > 6:
        fetch, write = sys.argv[5], sys.argv[6]
        calib = 1 << 30  # bytes of the calibration copy (1024 MiB read, 1024 MiB written)
        f_copy, w_copy = copy_value(fetch, "FETCH_SIZE"), copy_value(write, "WRITE_SIZE")
        f_scale = calib / (f_copy * 1024.0)
        w_scale = calib / (w_copy * 1024.0)
        f_k = per_dispatch(fetch, kernel, "FETCH_SIZE")
        w_k = per_dispatch(write, kernel, "WRITE_SIZE")
        hbm = f_k * 1024.0 * f_scale + w_k * 1024.0 * w_scale
        lines += ["", "## HBM traffic (PMC)", "",
                  "calibration copy (1 GiB read + 1 GiB written): FETCH_SIZE %.0f KiB -> scale %.3f; WRITE_SIZE %.0f KiB "
                  "-> scale %.3f" % (f_copy, f_scale, w_copy, w_scale),
                  "", "per dispatch: FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB" % (f_k, w_k),
                  "", "HBM bytes per launch (scaled): %.6e" % hbm]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
