"""Turns rocprofv3 CSV output (kernel stats, FETCH_SIZE / WRITE_SIZE counter
collections) into the short text summaries kept in profiles/, and
optionally the per-kernel HBM traffic file that bench.py reports.

usage: python paper_1102_3069_amd/prof/summarize.py <kernel_stats.csv>
           [fetch.csv write.csv copy_fetch.csv copy_write.csv copy_bytes [traffic.json]]
       python paper_1102_3069_amd/prof/summarize.py --busy <kernel_trace.csv> <pattern> <last_kernel> <count>
       python paper_1102_3069_amd/prof/summarize.py --counters <counter_collection.csv> [<pattern>]

--counters: the mean per dispatch of every counter of every kernel (whose
name contains <pattern>) in a counter-collection file.

--busy: over the last <count> intervals that end with a kernel whose name
contains <last_kernel> (one attempt of a batch each), the union of the
intervals of every kernel whose name contains <pattern> or <last_kernel>,
against the span and the sum of their durations (how busy the GPU was and
how much the launches overlapped).

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


def busy(path, pattern, last, count):
    rows = list(csv.DictReader(open(path)))
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows)
    ends = [i for i, x in enumerate(iv) if last in x[2]]
    if len(ends) < count + 1:
        raise SystemExit(f"only {len(ends)} kernels match {last!r}")
    first, end = ends[-count - 1] + 1, ends[-1] + 1
    sel = [x for x in iv[first:end] if pattern in x[2] or last in x[2]]
    t0, t1 = sel[0][0], max(e for _, e, _ in sel)
    union, cs, ce = 0, None, None
    for s_, e, _ in sel:
        if ce is None or s_ > ce:
            if ce is not None:
                union += ce - cs
            cs, ce = s_, e
        else:
            ce = max(ce, e)
    union += ce - cs
    total = sum(e - s_ for s_, e, _ in sel)
    print(f"{count} intervals, {len(sel)} kernels: span {(t1 - t0) / 1e3:.1f} us "
          f"({(t1 - t0) / 1e3 / count:.1f} us each), busy (union of kernel intervals) {union / 1e3:.1f} us "
          f"= {union / (t1 - t0):.3f} of the span, sum of kernel durations {total / 1e3:.1f} us "
          f"(overlap factor {total / union:.2f})")


def counters(path, pattern=""):
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        if pattern in r["Kernel_Name"]:
            d[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    for k, cs in d.items():
        means = ", ".join(f"{c} {sum(v) / len(v):.0f}" for c, v in sorted(cs.items()))
        print(f"* `{k[:90]}`: {means}")


if __name__ == "__main__":
    if len(sys.argv) in (3, 4) and sys.argv[1] == "--counters":
        counters(sys.argv[2], sys.argv[3] if len(sys.argv) == 4 else "")
    elif len(sys.argv) == 6 and sys.argv[1] == "--busy":
        busy(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]))
    else:
        main(sys.argv)
