"""Write a short text summary of a rocprofv3 --stats kernel table.

usage: python profiles/make_summary.py <kernel_stats.csv> <out.txt> "<title>" "<command>"
"""
import csv
import re
import sys


def main():
    src, dst, title, cmd = sys.argv[1:5]
    rows = list(csv.DictReader(open(src)))
    lines = ["# " + title, "#", "# command (one MI355X, repository root):", "#   " + cmd,
             "# durations in microseconds, from rocprofv3 --kernel-trace --stats", "",
             "%-26s %6s %12s %10s %7s" % ("kernel", "calls", "total_us", "avg_us", "pct")]
    for r in rows:
        name = re.sub(r"\(anonymous namespace\)::", "", r["Name"])
        name = re.sub(r"^void ", "", name).split("(")[0].split("::")[-1]
        lines.append("%-26s %6s %12.1f %10.1f %7.2f" % (name, r["Calls"], float(r["TotalDurationNs"]) / 1e3,
                                                         float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    open(dst, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
