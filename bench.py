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

Prints one JSON line.  "roofline" divides the algorithmic bytes of the
dominant kernel (what it must read and write: the magnetisation, the spectra,
the kernel spectrum, the fields; llg_kernel_bytes) by its mean duration, timed
by HIP events attached to each of its launches (the kernel's own execution,
as a profiler's kernel trace measures it; llg_profile_evals).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# the network's output unit: a coarse RK4 step of 1 ps lands ~1e-4 from the
# plain segment, so the correction is learned in units of 1e-4
SURROGATE_SCALE = 1e-4
METRIC = "cell-updates/s (H_eff evals) at 512x512x1 FP32"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--n", type=int, default=512, help="film side (cells)")
    ap.add_argument("--profile-evals", type=int, default=200)
    ap.add_argument("--cpu-baseline-evals", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default compiled variants")
    ap.add_argument("--evals-only", action="store_true",
                    help="run only the H_eff evaluations of the roofline measurement (for counter runs)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="worker processes of the all-cores CPU-baseline leg (0: every host core, at most 16)")
    ap.add_argument("--no-full-run", action="store_true", help="skip the 1 ns Dormand-Prince run of the film")
    ap.add_argument("--batch-separate", action="store_true",
                    help="batch: also time the same films as separate solvers, one after another")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30, help="copy: bytes per copy")
    ap.add_argument("--workload", choices=("film512", "film3d", "batch", "sp2", "surrogate", "table1", "copy"),
                    default="film512",
                    help="film512: the 512x512 film (the headline); film3d: the 256x256x64 periodic block "
                         "with the thermal field; batch: the 64-film sweep; "
                         "sp2: 200 relaxations shaped like the static standard problem, in one batch; "
                         "surrogate: train the learned proposer and time speculative verification; "
                         "table1: Euler step time over the film and cube sizes of the paper's Table 1; "
                         "copy: a plain device copy of --copy-bytes (HBM bandwidth, counter calibration)")
    ap.add_argument("--sur-traj", type=int, default=100, help="surrogate: training trajectories")
    ap.add_argument("--sur-pairs", type=int, default=200, help="surrogate: pairs per trajectory")
    ap.add_argument("--sur-epochs", type=float, default=4.0, help="surrogate: passes over the pairs")
    ap.add_argument("--sur-window", type=int, default=16, help="surrogate: proposals per round")
    ap.add_argument("--sur-held-out", type=int, default=8, help="surrogate: held-out trajectories")
    ap.add_argument("--sur-segments", type=int, default=200, help="surrogate: segments per held-out run")
    return ap.parse_args()


def host_description():
    """nproc, the cores this process may run on, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model}


def _oracle_evals(prob, m0, nevals, ready=None, go=None):
    """Worker of the CPU baseline: builds the oracle's kernel spectrum (not
    timed), then times nevals FP64 H_eff evaluations of m0."""
    import numpy as np
    from oracle import fields
    m = m0.astype(np.float64)
    fields.heff(m, prob)                  # builds and caches the oracle's kernel spectrum
    if ready is not None:
        ready.wait()                      # every worker has built its spectrum
        go.wait()
    t0 = time.perf_counter()
    for _ in range(nevals):
        fields.heff(m, prob)
    return time.perf_counter() - t0


def cpu_baseline(prob, m0, nevals, threads):
    """The FP64 oracle's H_eff evaluation timed on the host cores.  numpy's
    FFTs and array operations run on one thread, so the all-cores leg runs
    one oracle process per core (each with one BLAS/OpenMP thread), all
    evaluating the same film at once; the one-thread leg runs alone."""
    import multiprocessing as mp
    ncells = m0[0].size
    host = host_description()
    one = _oracle_evals(prob, m0, nevals)
    nproc = threads if threads > 0 else min(16, host["usable_cores"] or 1)
    per = max(2, nevals // 4)
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Manager() as mgr:
            ready, go = mgr.Barrier(nproc + 1), mgr.Barrier(nproc + 1)
            with ctx.Pool(nproc) as pool:
                res = [pool.apply_async(_oracle_evals, (prob, m0, per, ready, go)) for _ in range(nproc)]
                ready.wait()
                t0 = time.perf_counter()
                go.wait()
                [r.get() for r in res]
                wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    film = f"{prob['n'][0]}x{prob['n'][1]}x{prob['n'][2]}"
    return {"value": ncells * per * nproc / wall, "unit": "cell-updates/s", "cores": nproc, "kind": "oracle",
            "sample": f"{nproc} oracle processes (one thread each) x {per} FP64 H_eff evaluations of the "
                      f"{film} film, concurrently ({wall:.1f} s wall; kernel spectra built beforehand, not timed)",
            "host": host,
            "one_thread": {"value": ncells * nevals / one, "cores": 1,
                           "sample": f"{nevals} FP64 H_eff evaluations of the same film ({one:.1f} s)"}}


def copy_bandwidth(nbytes, reps=5):
    """GB/s (read + write) of a plain device-to-device copy of nbytes, timed
    with events on torch's current stream (the stream the copy runs on)."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, ms


def bench_copy(args):
    """A plain device copy of --copy-bytes, three dispatches: the measured
    HBM bandwidth, and the known-size kernel whose FETCH_SIZE / WRITE_SIZE
    counters calibrate the per-kernel traffic figures."""
    import torch
    n = args.copy_bytes // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    gbs, ms = copy_bandwidth(args.copy_bytes)
    print(json.dumps({"metric": "device copy bandwidth (read + write)", "value": gbs, "unit": "GB/s",
                      "n_gpus": 1, "ms_per_copy": ms, "bytes_per_copy": args.copy_bytes,
                      "peak": PEAK_HBM_GBS, "frac": gbs / PEAK_HBM_GBS}), flush=True)


# full template names of the 2D compiled-length kernels a film of padded
# lengths px x py runs with the (row, column) variant pair, per kernel kind
# of llg_profile_evals (zero-padded x: XPER false; 2D packed layout: NAT false)
def _kernel_name(kind, px, py, variants):
    import paper_1102_3069_amd as llg
    if variants is None:
        return None
    re_, rq = llg.variant_shape("row", px, variants[0])
    ce, cq = llg.variant_shape("col", py // 2, variants[1])
    return {"row_fwd": f"row_fwd_fast<{px}, {re_}, {rq}, false, false>",
            "spectral": f"col2d_fast<{py // 2}, {ce}, {cq}>",
            "row_inv": f"row_inv_fast<{px}, {re_}, {rq}, false, false>"}.get(kind)


# kernel names of the 3D path (256 x 256 x 64 block: x periodic of 256,
# y periodic of 256, z open of 2 x 64), per kernel kind
def _kernel_name_3d(kind):
    """Full template names of the 3D block's kernels (x periodic 256, the
    default variants; z open 64, y periodic 256)."""
    return {"row_fwd": "row_fwd_fast<256, 4, 2, true, true>", "spectral": "col3_tiled<64, 8, 4, 2, 3, 1>",
            "row_inv": "row_inv_fast<256, 4, 2, true, true>", "y_fwd": "col3_tiled<256, 16, 16, 1, 1, 0>",
            "y_inv": "col3_tiled<256, 16, 16, 1, 1, 2>"}.get(kind)


def measured_traffic(kind, prob, path=None, key=None, variants=None):
    """HBM bytes per launch of the kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary (scaled by a plain copy), or None when
    that summary was taken on other kernel sources or another size, or has
    no entry for the kernel's full template name."""
    import hashlib
    if path is None:
        path = os.path.join(ROOT, "profiles", f"film{prob['n'][0]}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    csrc = os.path.join(ROOT, "paper_1102_3069_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    if key is None:
        key = _kernel_name(kind, 2 * prob["n"][0], 2 * prob["n"][1], variants)
    for name, t in rec["kernels"].items():
        if key and key + "(" in name:
            return t["read_bytes"] + t["write_bytes"]
    return None


def tune_batch(b, args):
    """The batch's own autotuner (llg_batch_autotune): both compiled variants
    of every length its films use, timed on evaluations of all films; returns
    {"row 512": chosen variant, ...}."""
    if args.no_autotune:
        return {}
    return {f"{e['kind']} {e['length']}": e["variant"] for e in b.autotune(30)}


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
    tuned = tune_batch(b, args)
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
                      "films_done": int(sum(s["done"] for s in st1)),
                      "variants": tuned}}
    if args.batch_separate:
        b.close()
        out["config"]["separate_solvers"] = separate_solvers(llg, films, run, args.steps, wall)
    print(json.dumps(out), flush=True)


def separate_solvers(llg, films, run, attempts, batch_wall):
    """The same films as separate solvers advanced one after another, the
    same number of attempts each: the cost the grouped launches avoid."""
    import torch
    sols = []
    for p, m0 in films:
        s = llg.Solver(0)
        s.set_problem(p)
        s.set_m(m0)
        s.run_attempts(run["t_end"], run["tol"], run["dt0"], 10)
        sols.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sols:
        s.run_attempts(run["t_end"], run["tol"], s.stats()["dt_next"] or run["dt0"], attempts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s in sols:
        s.close()
    return {"ms_per_attempt_all_films": wall * 1e3 / attempts, "slower_than_batch": wall / batch_wall}


def bench_film3d(args):
    """The 256 x 256 x 64 block of 3 nm cubes, periodic in x and y (10
    images), 300 K thermal field, vortex start: fixed Heun steps of 5e-14 s
    (two H_eff evaluations each, the thermal draw held across both)."""
    import numpy as np
    import torch
    import paper_1102_3069_amd as llg
    import workloads
    llg.load()
    prob, m0, run = workloads.film_3d()
    ncells = int(np.prod(prob["n"]))
    s = llg.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    if args.evals_only:
        prof, total = s.profile_evals(args.profile_evals)
        print(json.dumps({"evals": args.profile_evals, "kernel_ms": prof, "eval_ms": total / args.profile_evals}))
        return
    steps = min(args.steps, 200)
    s.step("heun", run["dt"], max(1, min(args.warmup, 20)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step("heun", run["dt"], steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = ncells * 2 * steps / wall
    prof, prof_total = s.profile_evals(20)
    nbytes = s.kernel_bytes()
    dom = max(prof, key=lambda k: prof[k])
    achieved = nbytes[dom] / (prof[dom] * 1e-3) / 1e9
    eval_bytes = sum(nbytes.values())
    out = {"metric": "cell-updates/s (H_eff evals) at 256x256x64 FP32, periodic x/y, thermal", "value": value,
           "unit": "cell-updates/s", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 20),
           "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256x256x64 cells of 3 nm, periodic x and y (10 images), 300 K, vortex start, "
                                  "Heun steps of 5e-14 s (2 H_eff evals each)", "cells": ncells},
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": achieved / PEAK_HBM_GBS,
                        "traffic": measured_traffic(dom, prob, os.path.join(ROOT, "profiles", "block256x256x64_traffic.json"),
                                                    _kernel_name_3d(dom)),
                        "kernel_ms": prof, "kernel_bytes": nbytes,
                        "eval_ms": prof_total / 20,
                        "eval_frac": eval_bytes / (prof_total / 20 * 1e-3) / 1e9 / PEAK_HBM_GBS}}
    print(json.dumps(out), flush=True)


# GPU time per Euler step in the paper's Table 1 (GTX580, ms), context only
PAPER_TABLE1_MS = {(32, 32, 1): 0.59, (64, 64, 1): 0.60, (128, 128, 1): 0.69, (256, 256, 1): 1.11,
                   (512, 512, 1): 2.75, (1024, 1024, 1): 9.07, (2048, 2048, 1): 35.78, (8, 8, 8): 0.79,
                   (16, 16, 16): 1.03, (32, 32, 32): 1.70, (64, 64, 64): 5.52, (128, 128, 128): 35.42}


def bench_table1(args):
    """One Euler step (one H_eff evaluation, the torque and the update) over
    the sizes of the paper's Table 1: N x N films of 4 x 4 x 3 nm cells and
    N^3 cubes of 3 nm cells, random start, all deterministic terms."""
    import numpy as np
    import torch
    import paper_1102_3069_amd as llg
    import workloads
    llg.load()
    rows = []
    for n in list(PAPER_TABLE1_MS):
        prob, _ = workloads.small_problem(n=n, cell=(4e-9, 4e-9, 3e-9) if n[2] == 1 else (3e-9,) * 3, seed=1)
        m0 = workloads.random_unit(n, 2)
        dt = 1e-13 if n[2] == 1 else 2e-14
        rec = {"size": "x".join(map(str, n)), "paper_gpu_ms": PAPER_TABLE1_MS[n]}
        try:
            s = llg.Solver(0)
            s.set_problem(prob)
            s.set_m(m0)
            s.step("euler", dt, 5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step("euler", dt, 10)
            torch.cuda.synchronize()
            per = (time.perf_counter() - t0) / 10
            k = int(min(2000, max(10, 0.2 / per)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step("euler", dt, k)
            torch.cuda.synchronize()
            per = (time.perf_counter() - t0) / k
            rec.update(ms_per_step=per * 1e3, cell_updates_per_s=int(np.prod(n)) / per, steps=k)
            s.close()
        except llg.LLGError as err:
            rec["unsupported"] = str(err)
        rows.append(rec)
        print(json.dumps(rec), file=sys.stderr, flush=True)
    ref = [r for r in rows if r["size"] == "512x512x1"][0]
    out = {"metric": "Euler step time over the sizes of the paper's Table 1 (context)",
           "value": ref["cell_updates_per_s"], "unit": "cell-updates/s at 512x512x1", "n_gpus": 1,
           "steps": ref["steps"], "warmup": 5, "ms_per_step": ref["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "Euler steps, N x N films (4 x 4 x 3 nm) and N^3 cubes (3 nm), random start, "
                                  "demag + exchange + anisotropy + Zeeman", "table": rows}}
    print(json.dumps(out), flush=True)


def bench_sp2(args):
    """200 films of 5d x d x 0.1d (d/l_ex from 1 to 30, alpha = 1, demag and
    exchange only) relaxed from [1,1,1] saturation for 1 ns in one batch:
    per-film adaptive Dormand-Prince, grouped launches over all films.  The
    warm-up attempts are the sweep's first ones; the timed region runs the
    rest of the sweep until every film reached 1 ns."""
    import numpy as np
    import torch
    import paper_1102_3069_amd as llg
    import workloads
    llg.load()
    films, run = workloads.sp2_films()
    cells = np.array([int(np.prod(p["n"])) for p, _ in films])
    b = llg.Batch(films)
    t_tune = time.perf_counter()
    tuned = tune_batch(b, args)
    t_tune = time.perf_counter() - t_tune
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    st0 = b.run(run["t_end"], run["tol"], run["dt0"], max_attempts=max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st1 = b.run(run["t_end"], run["tol"], 0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    evals = np.array([s1["evals"] - s0["evals"] for s0, s1 in zip(st0, st1)])
    attempts = max(s["steps"] + s["rejected"] for s in st1) - max(s["steps"] + s["rejected"] for s in st0)
    value = float(np.sum(cells * evals)) / wall
    rem = {}
    for i in (0, 33, 66, 99, 133, 166, 199):
        m = b.get_m(i).reshape(3, -1).mean(axis=1)
        rem[f"{films[i][0]['d_over_lex']:.2f}"] = [round(float(m[0]), 4), round(float(m[1]), 4)]
    out = {"metric": "cell-updates/s (H_eff evals), 200-film relaxation sweep", "value": value,
           "unit": "cell-updates/s", "n_gpus": 1, "steps": int(attempts), "warmup": args.warmup,
           "ms_per_step": wall * 1e3 / max(attempts, 1), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "200 films of 5d x d x 0.1d, d/l_ex 1..30 (ny = 2 d/l_ex cells across, "
                                  "4..60; nx = 5 ny), alpha 1, demag + exchange, from [1,1,1] to 1 ns, "
                                  "adaptive Dormand-Prince per film, grouped launches",
                      "cells": int(cells.sum()), "evals_max": int(evals.max()),
                      "sweep_s": t1 - t_start, "films_done": int(sum(s["done"] for s in st1)),
                      "remanence_mx_my": rem, "tuning_s": t_tune, "variants": tuned,
                      "paper_context": "GTX580: 200 separate runs in 3 min 21 s (Sec. 4.1)"}}
    print(json.dumps(out), flush=True)


def bench_surrogate(args):
    """The learned surrogate on 256 x 256 films: solver-generated pairs,
    training on the MFMA kernels, then the held-out trajectories advanced by
    plain RK4 and by speculative verification on the same GPU."""
    import numpy as np
    import torch
    import paper_1102_3069_amd as llg
    import workloads
    from paper_1102_3069_amd import surrogate_train as tr
    llg.load()
    n = 256
    films, run = workloads.surrogate_films(args.sur_traj, seed=5, n_side=n)
    t0 = time.perf_counter()
    X, E, B = tr.generate_pairs(llg, films, run, pairs_per_traj=args.sur_pairs)
    t_data = time.perf_counter() - t0
    npairs = X.shape[0] * (X.shape[1] - 1)
    batch = 16
    steps = int(args.sur_epochs * npairs / batch)
    sur = llg.Surrogate(n, n, max_batch=batch)
    sur.set_params(workloads.surrogate_init(0))
    sur.set_output_scale(SURROGATE_SCALE)
    res = tr.train(sur, X, B, steps=steps, batch=batch, lr0=2e-3, E=E)
    del X, E
    torch.cuda.empty_cache()
    train_flops = 236.7e3 * n * n * steps * batch
    # ablation: the same proposals without the network (all weights zero, so
    # dm = 0: the plain solver's one coarse RK4 step of the whole segment),
    # on the same object with its parameters swapped, interleaved with the
    # network's runs threshold by threshold
    trained = sur.get_params()
    zeros = np.zeros_like(trained)
    held, _ = workloads.surrogate_films(args.sur_held_out, seed=6, n_side=n)
    thresholds = (1e-2, 1e-4, 5e-5, 2e-5)
    t_plain = 0.0
    runs = {(kind, th): {"t": 0.0, "dev": 0.0, "stats": []} for kind in ("net", "bare") for th in thresholds}
    for prob, m0 in held:
        s = llg.Solver(0)
        s.set_problem(prob)
        s.set_m(m0)
        s.step("rk4", run["dt"], run["burn_in"])
        m_start = s.get_m()
        s.set_m(m_start)
        t0 = time.perf_counter()
        s.step("rk4", run["dt"], run["seg_steps"] * args.sur_segments)
        t_plain += time.perf_counter() - t0
        m_plain = s.get_m()
        sur.advance(prob, m_start, n_segments=1, window=args.sur_window, dt=run["dt"])   # builds the batches
        for th in thresholds:
            for kind, params in (("net", trained), ("bare", zeros)):
                sur.set_params(params)
                r = runs[(kind, th)]
                t0 = time.perf_counter()
                m_s, st = sur.advance(prob, m_start, n_segments=args.sur_segments, window=args.sur_window,
                                      dt=run["dt"], max_dm=th)
                r["t"] += time.perf_counter() - t0
                r["stats"].append(st)
                r["dev"] = max(r["dev"], float(np.max(np.linalg.norm((m_s - m_plain).reshape(3, -1), axis=0))))

    def summary(kind, th):
        r = runs[(kind, th)]
        acc = sum(x["accepted"] for x in r["stats"]) / max(1, sum(x["proposals"] for x in r["stats"]))
        return {"speedup": t_plain / r["t"], "acceptance": acc,
                "max_dm_accepted": max(x["max_dm_accepted"] for x in r["stats"]),
                "max_dm_seen": max(x["max_dm_seen"] for x in r["stats"]), "end_to_end_max_dev": r["dev"]}
    segs = args.sur_held_out * args.sur_segments
    th0 = thresholds[0]
    head = summary("net", th0)
    # at 1e-2 both arms accept every proposal and do the same work: that
    # speedup belongs to the scheme (time-parallel verification of
    # coarse-step proposals); the network's own gain is the ratio of the
    # arms where their acceptance differs
    gain = {f"{th:g}": summary("net", th)["speedup"] / summary("bare", th)["speedup"] for th in thresholds}
    out = {"metric": "speedup of speculative verification over plain RK4 at max |dm| <= 1e-2",
           "value": head["speedup"], "unit": "x", "n_gpus": 1, "steps": segs, "warmup": 1,
           "ms_per_step": runs[("net", th0)]["t"] * 1e3 / segs, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16 (network), f32 (solver)", "data": "synthetic",
           "config": {"workload": f"{args.sur_held_out} held-out 256x256 films, {args.sur_segments} segments of "
                                  f"10 RK4 steps (dt 1e-13 s), window {args.sur_window}; proposals "
                                  "normalize(one RK4 step of the whole segment + network correction)",
                      "plain_s": t_plain, "speculative_s": runs[("net", th0)]["t"], **head,
                      "speedup_source": "at 1e-2 every proposal of both arms is accepted: the speedup comes from "
                                        "speculative verification of coarse-step proposals, not from the network; "
                                        "network_gain_over_bare gives the network's own share per threshold",
                      "network_gain_over_bare": gain,
                      "thresholds": {f"{th:g}": {"network": summary("net", th), "without_network": summary("bare", th)}
                                     for th in thresholds},
                      "train_pairs": npairs, "train_steps": steps,
                      "train_batch": batch, "final_loss": float(np.mean(res["losses"][-50:])),
                      "train_px_per_s": res["px_per_s"],
                      "train_tflops": train_flops / res["wall_s"] / 1e12, "data_gen_s": t_data}}
    print(json.dumps(out), flush=True)


def model_bytes_2d(n, px, py):
    """Algorithmic bytes of one H_eff evaluation of an n[0] x n[1] film on a
    px x py FFT grid (FP32): read m and write H, the kernel spectrum read
    once, and one write + read round trip of the half spectrum for each of
    the two exchanges between the x and y directions."""
    cells = n[0] * n[1]
    spec = 3 * 8 * (px // 2 + 1) * n[1]
    kern = 4 * 4 * (px // 2 + 1) * (py // 2 + 1)
    return 2 * 12 * cells + 2 * 2 * spec + kern


def full_run(llg, prob, m0, run):
    """The film from its start state to 1 ns with adaptive Dormand-Prince
    (tolerance 1e-5): wall time and the work the controller did."""
    import numpy as np
    import torch
    s = llg.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    s.run(2e-12, run["tol"], run["dt0"])           # captures the attempt graph
    s.set_m(m0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.run(run["t_end"], run["tol"], run["dt0"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m = s.get_m().reshape(3, -1).mean(axis=1)
    s.close()
    return {"t_end_s": run["t_end"], "wall_s": wall, "evals": st["evals"], "accepted": st["steps"],
            "rejected": st["rejected"], "cell_updates_per_s": int(np.prod(prob["n"])) * st["evals"] / wall,
            "mean_m": [round(float(v), 5) for v in m]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the path is measured on one GPU's "
              "share; a film split over several GPUs needs an all-to-all transpose around the spectral pass, "
              "which is not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload in ("batch", "sp2", "film3d", "table1", "copy"):
        return {"batch": bench_batch, "sp2": bench_sp2, "film3d": bench_film3d,
                "table1": bench_table1, "copy": bench_copy}[args.workload](args)
    import numpy as np
    import torch
    import paper_1102_3069_amd as llg
    import workloads

    llg.load()
    prob, m0, run = workloads.film_512(args.n)
    ncells = int(np.prod(prob["n"]))
    # the CPU leg first, before this process touches the GPU (its worker
    # processes are started fresh)
    cpu = None
    if not args.no_cpu_baseline and not args.evals_only:
        cpu = cpu_baseline(prob, m0, args.cpu_baseline_evals, args.cpu_threads)
    s = llg.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    # compiled-variant choice for these FFT lengths: the timed workload's own
    # step (50 Dormand-Prince attempts from the start state per pair, the
    # state kept); the evaluation-only runs tune on H_eff evaluations
    tune_kind = "eval_ms" if args.evals_only else "attempt_ms"
    if args.no_autotune:
        tune_ms, tune_choice = {}, None
    elif args.evals_only:
        tune_ms, tune_choice = s.autotune(50)
    else:
        tune_ms, tune_choice = s.autotune_attempts(run["tol"], run["dt0"], 50)
    variants = s.get_variants()
    s.set_m(m0)
    if args.evals_only:
        prof, total = s.profile_evals(args.profile_evals)
        print(json.dumps({"evals": args.profile_evals, "kernel_ms": prof, "eval_ms": total / args.profile_evals,
                          "variants": variants}))
        return
    # warm-up attempts (they also capture the graph)
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

    # per-kernel durations (HIP events attached to each kernel's launch on
    # the library's stream) and the algorithmic bytes of each kernel kind
    prof, prof_total = s.profile_evals(args.profile_evals)
    nbytes = s.kernel_bytes()
    dom = max(prof, key=lambda k: prof[k])
    achieved = nbytes[dom] / (prof[dom] * 1e-3) / 1e9
    px, py = 2 * prob["n"][0], 2 * prob["n"][1]
    eval_bytes = model_bytes_2d(prob["n"], px, py)
    copy_gbs, _ = copy_bandwidth(1 << 30)
    eval_gbs = eval_bytes * value / ncells / 1e9
    roofline = {"bound": "hbm", "kernel": _kernel_name(dom, px, py, variants) or dom, "achieved": achieved,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": measured_traffic(dom, prob, variants=variants),
                "kernel_ms": prof, "kernel_bytes": nbytes,
                "eval_ms": prof_total / args.profile_evals,
                "eval_model_bytes": eval_bytes, "eval_gbs": eval_gbs, "eval_frac": eval_gbs / PEAK_HBM_GBS,
                "copy_gbs": copy_gbs, "eval_frac_of_copy": eval_gbs / copy_gbs}
    s.close()
    config = {"workload": f"thin film {prob['n'][0]}x{prob['n'][1]}x1, 4x4x3 nm cells, "
                          "adaptive Dormand-Prince 5(4) attempts (6 H_eff evals each) toward 1 ns",
              "cells": ncells, "evals": evals, "sim_time_s": st1["t"],
              "variants": {"chosen": list(variants),
                           tune_kind: {f"{r}{c}": round(v, 5) for (r, c), v in tune_ms.items()}},
              "paper_context": "GTX580 Euler step at 512^2: 9.53e7 cell-updates/s (Table 1)"}
    if not args.no_full_run:
        config["full_run_1ns"] = full_run(llg, prob, m0, run)
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": attempts, "warmup": args.warmup, "ms_per_step": wall * 1e3 / max(attempts, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": config, "roofline": roofline,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
