"""Benchmark of the effective-field evaluation and time step on one MI355X.

Workload: the 512 x 512 x 1 thin film (4 x 4 x 3 nm cells, Ms 8e5 A/m,
A 1.3e-11 J/m, alpha 0.02, uniaxial 5e3 J/m^3 along x, 25 mT at 170 deg)
integrated with adaptive Dormand-Prince 5(4) toward 1 ns.  One step is one
attempted adaptive step: six H_eff evaluations (FFT convolution with the
demag kernel, exchange, anisotropy and Zeeman terms), the LL torque, the
stage combinations, the embedded error estimate and the device-side step
controller, replayed from a captured HIP graph.  The metric counts
cell-updates = cells x H_eff evaluations per second, with all inputs already
resident in HBM.

Prints one JSON line; see DESIGN.md for the byte model behind "roofline".
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "cell-updates/s (H_eff evals) at 512x512x1 FP32"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--n", type=int, default=512, help="film side (cells)")
    ap.add_argument("--profile-evals", type=int, default=200)
    ap.add_argument("--cpu-baseline-evals", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("film512", "batch"), default="film512",
                    help="film512: the 512x512 film (the headline); batch: the 64-film sweep")
    return ap.parse_args()


def cpu_baseline(prob, m0, nevals):
    """The FP64 oracle's H_eff evaluation timed on the host (numpy; its FFTs
    and array operations run on one thread)."""
    import numpy as np
    from oracle import fields
    m = m0.astype(np.float64)
    fields.heff(m, prob)                  # builds and caches the oracle's kernel spectrum
    t0 = time.perf_counter()
    for _ in range(nevals):
        fields.heff(m, prob)
    dt = time.perf_counter() - t0
    ncells = m0[0].size
    return {"value": ncells * nevals / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{nevals} FP64 H_eff evaluations of the same {prob['n'][0]}x{prob['n'][1]}x1 film "
                      f"({dt:.1f} s; kernel spectrum built beforehand, not timed)"}


def bench_batch(args):
    """64 independent films of uneven size (sides 64..256) advanced together:
    one grouped launch per pass over all films, per-film adaptive steps."""
    import numpy as np
    import torch
    import paper_1102_3069_amd as llg
    import workloads
    llg.load()
    films, run = workloads.film_batch()
    cells = np.array([int(np.prod(p["n"])) for p, _ in films])
    b = llg.Batch(films)
    st0 = b.run(run["t_end"], run["tol"], run["dt0"], max_attempts=max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st1 = b.run(run["t_end"], run["tol"], run["dt0"], max_attempts=args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals = np.array([s1["evals"] - s0["evals"] for s0, s1 in zip(st0, st1)])
    value = float(np.sum(cells * evals)) / wall
    out = {"metric": "cell-updates/s (H_eff evals), 64-film batch", "value": value, "unit": "cell-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "64 films, sides from {64,96,128,192,256}, adaptive Dormand-Prince, "
                                  "grouped launches over all films", "cells": int(cells.sum()),
                      "films_done": int(sum(s["done"] for s in st1))}}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.workload == "batch":
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        return bench_batch(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is "
              "described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1102_3069_amd as llg
    import workloads

    llg.load()
    prob, m0, run = workloads.film_512(args.n)
    ncells = int(np.prod(prob["n"]))
    s = llg.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    # warm-up attempts (also builds the demag kernel and captures the graph)
    s.run_attempts(run["t_end"], run["tol"], run["dt0"], max(1, args.warmup))
    st0 = s.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st1 = s.run_attempts(run["t_end"], run["tol"], st0["dt_next"] or run["dt0"], args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals = st1["evals"] - st0["evals"]
    attempts = (st1["steps"] + st1["rejected"]) - (st0["steps"] + st0["rejected"])
    value = ncells * evals / wall

    # per-kernel durations (HIP events on the library's stream) and the
    # algorithmic bytes of each kernel kind
    prof, prof_total = s.profile_evals(args.profile_evals)
    nbytes = s.kernel_bytes()
    dom = max(prof, key=lambda k: prof[k])
    achieved = nbytes[dom] / (prof[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "kernel_ms": prof, "kernel_bytes": nbytes,
                "eval_ms": prof_total / args.profile_evals}

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": attempts, "warmup": args.warmup, "ms_per_step": wall * 1e3 / max(attempts, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"thin film {prob['n'][0]}x{prob['n'][1]}x1, 4x4x3 nm cells, "
                               "adaptive Dormand-Prince 5(4) attempts (6 H_eff evals each) toward 1 ns",
                   "cells": ncells, "evals": evals, "sim_time_s": st1["t"],
                   "paper_context": "GTX580 Euler step at 512^2: 9.53e7 cell-updates/s (Table 1)"},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, m0, args.cpu_baseline_evals)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
