"""Condense a rocprofv3 kernel-stats CSV into a short text table.

Usage: python -m paper_1504_02264_amd.profsum <run_kernel_stats.csv> [title] [command]
"""
import csv
import sys


def main():
    path = sys.argv[1]
    title = sys.argv[2] if len(sys.argv) > 2 else path
    cmd = sys.argv[3] if len(sys.argv) > 3 else ""
    rows = list(csv.DictReader(open(path)))
    print(f"# {title}")
    if cmd:
        print(f"command: {cmd}")
    print(f"{'kernel':44s} {'calls':>8s} {'avg_us':>9s} {'min_us':>9s} {'total_ms':>10s} {'pct':>6s}")
    for r in rows:
        name = r["Name"].replace("les::(anonymous namespace)::", "").replace("void ", "")
        name = name.split("(")[0]
        print(f"{name:44s} {int(r['Calls']):8d} {float(r['AverageNs']) / 1e3:9.2f} "
              f"{float(r['MinNs']) / 1e3:9.2f} {float(r['TotalDurationNs']) / 1e6:10.2f} "
              f"{float(r['Percentage']):6.2f}")


if __name__ == "__main__":
    main()
