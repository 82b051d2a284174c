"""Turns rocprofv3 CSV output (kernel stats, FETCH_SIZE / WRITE_SIZE counter
collections) into the short text summaries kept in this folder.

usage: python paper_1102_3069_amd/prof/summarize.py <kernel_stats.csv> [fetch.csv write.csv
       copy_fetch.csv copy_write.csv copy_bytes]
"""
import collections
import csv
import sys


def stats(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["Percentage"])))
    return out


def counter_means(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in d.items()}


def main(argv):
    print("kernel | calls | avg us | % time")
    for name, calls, avg, pct in stats(argv[1])[:12]:
        print(f"{name[:90]} | {calls} | {avg / 1000:.2f} | {pct:.1f}")
    if len(argv) >= 7:
        fetch, write = counter_means(argv[2]), counter_means(argv[3])
        cf, cw = counter_means(argv[4]), counter_means(argv[5])
        copy_bytes = float(argv[6])
        copy = [k for k in cf if "copyBuffer" in k][0]
        f_scale = copy_bytes / (cf[copy] * 1024.0)
        w_scale = copy_bytes / (cw[copy] * 1024.0)
        print(f"\ncalibration: plain copy of {copy_bytes:.0f} B reads FETCH_SIZE {cf[copy]:.1f} KiB, "
              f"WRITE_SIZE {cw[copy]:.1f} KiB -> scale fetch x{f_scale:.3f}, write x{w_scale:.3f}")
        print("\nkernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled MB read | scaled MB written")
        for k in fetch:
            if k in write and ("llg::" in k):
                print(f"{k[:90]} | {fetch[k]:.1f} | {write[k]:.1f} | "
                      f"{fetch[k] * 1024 * f_scale / 1e6:.3f} | {write[k] * 1024 * w_scale / 1e6:.3f}")


if __name__ == "__main__":
    main(sys.argv)
