"""Summaries of rocprofv3 output for the benchmark's roofline.

    python -m paper_1402_5670_amd.profiling traffic FETCH.csv WRITE.csv OUT.json
    python -m paper_1402_5670_amd.profiling stats KERNEL_STATS.csv

`traffic` turns two counter-collection runs (FETCH_SIZE, then WRITE_SIZE, in
KiB per dispatch) into bytes per launch for every kernel.  Each counter is
scaled by what it reads for the device-to-device copy in the same run (one
copy of a known size, `bench.py --calib-copy-mib`).  The JSON records a hash
of the kernel sources: bench.py reports the traffic only while the kernels
are unchanged.
"""
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))


TRANSFORM_SOURCES = ("kernels2d.hip", "kernels3d.hip", "fft_core.hpp", "dispatch.hpp")


def source_hash():
    """Hash of the transform kernel sources the traffic summary describes."""
    h = hashlib.sha256()
    for path in sorted(os.path.join(PKG, "csrc", f) for f in TRANSFORM_SOURCES):
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(k):
    k = k.replace("(anonymous namespace)::", "")
    return k.split("(")[0].replace("void ", "").strip()


def _counter(path, name):
    vals = defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") == name:
                vals[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_csv, write_csv, calib_mib=1024, calib_kernel="__amd_rocclr_copyBuffer"):
    f = _counter(fetch_csv, "FETCH_SIZE")
    w = _counter(write_csv, "WRITE_SIZE")
    calib = calib_mib * 1024.0           # KiB the copy really reads and writes
    ff = calib / max(f[calib_kernel])
    fw = calib / max(w[calib_kernel])
    out = {"source_hash": source_hash(), "fetch_scale": ff, "write_scale": fw, "kernels": {}}
    for k in f:
        if k == calib_kernel:
            continue
        # the most frequent launch shape dominates: use the median launch
        fr = sorted(f[k])[len(f[k]) // 2] * ff * 1024.0
        wr = sorted(w.get(k, [0.0]))[len(w.get(k, [0.0])) // 2] * fw * 1024.0
        out["kernels"][k] = {"read_bytes": fr, "write_bytes": wr, "launches": len(f[k])}
    return out


def stats_table(stats_csv):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["| Kernel | Calls | Total ms | Avg us | % |", "|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | "
                     f"{int(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.2f} |")
    return "\n".join(lines)


def main(argv):
    if argv[:1] == ["traffic"]:
        res = traffic(argv[1], argv[2])
        with open(argv[3], "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res, indent=1))
    elif argv[:1] == ["stats"]:
        print(stats_table(argv[1]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
