"""Condense rocprofv3 output into the short text summaries kept in profiles/.

  python -m paper_1504_02264_amd.profsum stats <run_kernel_stats.csv> <title> <command>
      per-kernel call count and durations of a --kernel-trace --stats run

  python -m paper_1504_02264_amd.profsum pmc <fetch.csv> <write.csv> <calib_MiB> <title> <command>
      per-kernel HBM bytes per dispatch from a FETCH_SIZE run and a WRITE_SIZE
      run, each scaled by what the same counter reads for the plain copy of
      calib_MiB MiB that the profiled command also runs; records the SHA-256
      of the SOR kernel sources so a reader can tell whether the kernel has
      changed since the counters were taken
"""
import collections
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOR_SOURCES = ("csrc/sor_bodies.h", "csrc/kernels_sor.hip")


def sor_source_hash() -> str:
    h = hashlib.sha256()
    for rel in SOR_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)", "anon").replace("void ", "")
    name = name.replace("les::net::anon::", "").replace("les::anon::", "")
    return name.split("(")[0].strip()


def stats(path, title, cmd):
    rows = list(csv.DictReader(open(path)))
    print(f"# {title}")
    print(f"command: {cmd}")
    print(f"{'kernel':44s} {'calls':>8s} {'avg_us':>9s} {'min_us':>9s} {'total_ms':>10s} {'pct':>6s}")
    for r in rows:
        print(f"{short(r['Name']):44s} {int(r['Calls']):8d} {float(r['AverageNs']) / 1e3:9.2f} "
              f"{float(r['MinNs']) / 1e3:9.2f} {float(r['TotalDurationNs']) / 1e6:10.2f} "
              f"{float(r['Percentage']):6.2f}")


def _per_kernel(path):
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(list)
    copy_max = 0.0
    for r in rows:
        v = float(r["Counter_Value"])
        k = short(r["Kernel_Name"])
        agg[k].append(v)
        if "copyBuffer" in k:
            copy_max = max(copy_max, v)
    return agg, copy_max


def pmc(fetch_csv, write_csv, calib_mib, title, cmd):
    fa, fcopy = _per_kernel(fetch_csv)
    wa, wcopy = _per_kernel(write_csv)
    calib_kib = float(calib_mib) * 1024.0
    ff = calib_kib / fcopy if fcopy else float("nan")
    wf = calib_kib / wcopy if wcopy else float("nan")
    print(f"# {title}")
    print(f"command: {cmd}")
    print(f"copy calibration: {calib_mib} MiB copy reads FETCH_SIZE {fcopy:.1f} KiB -> factor {ff:.4f}; "
          f"WRITE_SIZE {wcopy:.1f} KiB -> factor {wf:.4f}")
    print(f"sor_source_sha256: {sor_source_hash()}")
    print(f"{'kernel':30s} {'dispatches':>10s} {'fetch_bytes':>14s} {'write_bytes':>14s}")
    for k in sorted(fa):
        if k not in wa:
            continue
        fb = sum(fa[k]) / len(fa[k]) * 1024.0 * ff
        wb = sum(wa[k]) / len(wa[k]) * 1024.0 * wf
        print(f"{k:30s} {len(fa[k]):10d} {fb:14.0f} {wb:14.0f}")


def read_traffic(path, kernel):
    """(fetch_bytes, write_bytes) per dispatch of kernel from a pmc summary,
    or None if the summary is missing or the SOR sources changed since."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"sor_source_sha256: ([0-9a-f]+)", txt)
    if not m or m.group(1) != sor_source_hash():
        return None
    for line in txt.splitlines():
        parts = line.rsplit(None, 3)
        if len(parts) == 4 and parts[0] == kernel:
            return float(parts[2]), float(parts[3])
    return None


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6])
    else:
        raise SystemExit(__doc__)
