"""Turns rocprofv3 CSV output (kernel stats, FETCH_SIZE / WRITE_SIZE counter
collections) into the short text summaries kept in profiles/, and
optionally the per-kernel HBM traffic file that bench.py reports.

usage: python paper_1102_3069_amd/prof/summarize.py <kernel_stats.csv>
           [fetch.csv write.csv copy_fetch.csv copy_write.csv copy_bytes [traffic.json]]

The plain copy of `bench.py --workload copy` moves copy_bytes per dispatch; the ratio of
that to what its counters read is the scale applied to every kernel.  The
traffic file records, per kernel name, the scaled bytes read and written per
dispatch and a hash of the HIP sources the library was built from, so that
bench.py can tell when the counters no longer describe the current kernels.
"""
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "csrc")


def source_hash():
    """SHA-256 over the HIP sources and headers of the library."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def stats(path):
    rows = list(csv.DictReader(open(path)))
    return [(r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["Percentage"])) for r in rows]


def counter_means(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in d.items()}


def main(argv):
    print("kernel | calls | avg us | % time")
    for name, calls, avg, pct in stats(argv[1])[:14]:
        print(f"{name[:100]} | {calls} | {avg / 1000:.2f} | {pct:.1f}")
    if len(argv) >= 7:
        fetch, write = counter_means(argv[2]), counter_means(argv[3])
        cf, cw = counter_means(argv[4]), counter_means(argv[5])
        copy_bytes = float(argv[6])
        copy = [k for k in cf if "copyBuffer" in k][0]
        f_scale = copy_bytes / (cf[copy] * 1024.0)
        w_scale = copy_bytes / (cw[copy] * 1024.0)
        print(f"\ncalibration: a plain copy of {copy_bytes:.0f} B per dispatch reads FETCH_SIZE {cf[copy]:.1f} KiB, "
              f"WRITE_SIZE {cw[copy]:.1f} KiB -> scale fetch x{f_scale:.3f}, write x{w_scale:.3f}")
        print("\nkernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled MB read | scaled MB written")
        traffic = {}
        for k in fetch:
            if k in write and "llg::" in k:
                rd, wr = fetch[k] * 1024 * f_scale, write[k] * 1024 * w_scale
                traffic[k] = {"read_bytes": rd, "write_bytes": wr}
                print(f"{k[:100]} | {fetch[k]:.1f} | {write[k]:.1f} | {rd / 1e6:.3f} | {wr / 1e6:.3f}")
        if len(argv) >= 8:
            with open(argv[7], "w") as f:
                json.dump({"source_sha256": source_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
                           "kernels": traffic}, f, indent=1)


if __name__ == "__main__":
    main(sys.argv)
