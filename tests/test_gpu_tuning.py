"""Compiled variants of the 2D kernels and the autotuner: every (row,
column) variant pair gives H_eff within the FP32 bar of the FP64 oracle,
the autotuner times all pairs and keeps one, and batched films follow the
table bit for bit like single films."""
import numpy as np
import pytest

import workloads
from oracle import fields as ofields

pytestmark = pytest.mark.gpu

# (nx, ny): row lengths Px = 2 nx and column half lengths Py / 2 = ny that
# have compiled variants, several tiles and both even and 3-smooth sizes
SIZES = [(32, 32), (64, 96), (96, 64), (128, 192), (192, 128), (256, 32), (384, 96), (512, 64), (1024, 32),
         (32, 1024)]


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(3, -1)
    b = np.asarray(b, dtype=np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


@pytest.fixture
def reset_table(lib):
    made = []
    yield made
    for s in made:           # back to variant 0 for the lengths these solvers touched
        s.set_variants(0, 0)


@pytest.mark.parametrize("n", SIZES)
def test_every_variant_matches_oracle(lib, n, reset_table):
    prob, m0 = workloads.small_problem((n[0], n[1], 1), seed=n[0] + n[1])
    ref = ofields.heff(m0.astype(np.float64), prob)
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    reset_table.append(s)
    tried = 0
    for rv in range(2):
        for cv in range(2):
            try:
                s.set_variants(rv, cv)
            except lib.LLGError as err:
                # a variant whose LDS would not fit this geometry is refused
                assert err.code == lib.LLG_E_ARG and (rv, cv) != (0, 0)
                print(f"{n} variants ({rv}, {cv}): refused", flush=True)
                continue
            e = maxrel(s.eval_heff(), ref)
            print(f"{n} variants ({rv}, {cv}): {e:.2e}", flush=True)
            assert e <= 1e-5
            tried += 1
    assert tried >= 2


def test_autotune_times_all_pairs(lib, reset_table):
    prob, m0, _ = workloads.film_512(512)
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    reset_table.append(s)
    ms, choice = s.autotune(10)
    print("autotune 512x512:", ms, "->", choice, flush=True)
    assert all(v > 0 for v in ms.values())
    assert ms[choice] == min(ms.values())
    ref = ofields.heff(m0.astype(np.float64), prob)
    assert maxrel(s.eval_heff(), ref) <= 1e-5


def test_autotune_attempts_keeps_the_state(lib, default_variants):
    """The attempt-timed tuner (Sec. 2.2's adaptive Dormand-Prince, the
    benchmarked step) times every pair, keeps the fastest, and leaves m,
    time, controller, statistics and attempt log as they were; the run that
    follows equals, bit for bit, a fresh solver restored to the same state
    with the chosen pair."""
    prob, m0, run = workloads.film_512(512)
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    s.run_attempts(run["t_end"], run["tol"], run["dt0"], 3)
    st0, mb = s.get_state()
    log0 = s.attempts()
    ms, choice = s.autotune_attempts(run["tol"], 0.0, 8)
    print("autotune_attempts 512x512:", ms, "->", choice, flush=True)
    assert all(v > 0 for v in ms.values())
    assert ms[choice] == min(ms.values())
    assert s.get_variants() == choice
    st1, ma = s.get_state()
    assert st1 == st0
    assert np.array_equal(ma, mb)
    assert s.attempts() == log0
    s.run_attempts(run["t_end"], run["tol"], 0.0, 4)
    f = lib.Solver(0)
    f.set_problem(prob)
    f.set_state(st0, mb)
    f.set_variants(*choice)
    f.run_attempts(run["t_end"], run["tol"], 0.0, 4)
    assert np.array_equal(s.get_m(), f.get_m())
    assert s.stats()["t"] == f.stats()["t"]
    with pytest.raises(lib.LLGError):
        s.autotune_attempts(run["tol"], 0.0, 0)
    s.close()
    f.close()


def test_batch_follows_the_table(lib, reset_table):
    rng = np.random.default_rng(3)
    films = []
    for side in (64, 96, 128):
        prob, _ = workloads.small_problem((side, side, 1), seed=side)
        films.append((prob, workloads.random_unit((side, side, 1), int(rng.integers(1 << 30)))))
    singles = []
    for prob, m0 in films:
        s = lib.Solver(0)
        s.set_problem(prob)
        s.set_m(m0)
        s.set_variants(1, 1)
        reset_table.append(s)
        singles.append(s)
    b = lib.Batch(films)
    b.step("rk4", 1e-13, 5)
    for i, s in enumerate(singles):
        s.step("rk4", 1e-13, 5)
        assert np.array_equal(b.get_m(i), s.get_m()), f"film {i}"


@pytest.mark.parametrize("shape", [(64, 64, 1), (32, 32, 16)])
def test_profile_evals_times_each_kernel(lib, shape):
    """llg_profile_evals: every pass of the evaluation gets a positive
    kernel time (2D: three kernels; 3D: five), none longer than an
    evaluation's wall time, and together about that wall time (consecutive
    kernels overlap their start and drain a little, so the sum may exceed
    it slightly on tiny grids)."""
    prob, m0 = workloads.small_problem(shape, seed=5)
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    prof, total = s.profile_evals(10)
    per = total / 10
    print(shape, {k: round(v * 1e3, 2) for k, v in prof.items()}, "eval", round(per * 1e3, 2), flush=True)
    want = ("row_fwd", "spectral", "row_inv") + (("y_fwd", "y_inv") if shape[2] > 1 else ())
    assert all(prof[k] > 0 for k in want)
    assert all(prof[k] == 0 for k in prof if k not in want)
    assert all(prof[k] <= per for k in want)
    assert sum(prof.values()) <= per * 1.25
    s.close()
