"""Parity with the FP64 oracle at the shapes and launch configurations the
benchmarks run: the 512 x 512 film's Dormand-Prince attempts on the tuned
variant pair, the 3D block's kernels (256-point periodic rows in the natural
layout, 64-point periodic y, 128-point open z) on a grid the oracle
evaluates in seconds, every compiled variant on ragged films (nx < Px / 2,
ny < Py / 2) in evaluation and in stage mode, and solvers that keep their
own variants whatever another solver tunes."""
import sys

import numpy as np
import pytest

import workloads
from oracle import fields, llg as ollg

pytestmark = pytest.mark.gpu


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(3, -1)
    b = np.asarray(b, dtype=np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


def note(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def solver(lib, prob, m0):
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    return s


def test_dp45_512_tuned_pair_replay(lib, default_variants):
    """The benchmark's path: the 512 x 512 film, the autotuner's variant pair
    (as bench.py picks it), three adaptive Dormand-Prince attempts replayed
    by the oracle (19 FP64 evaluations) to 1e-5; then the same on the pair
    the tuner did not pick first (both row variants covered)."""
    prob, m0, run = workloads.film_512(512)
    s = solver(lib, prob, m0)
    ms, choice = s.autotune(5)
    note("case: 512x512 film, tuned pair", choice, ms)
    pairs = [choice, (1 - choice[0], 1 - choice[1])]
    for rv, cv in pairs:
        s.set_variants(rv, cv)
        s.set_m(m0)
        st = s.run_attempts(run["t_end"], run["tol"], run["dt0"], 3)
        log = s.attempts()
        assert len(log) == 3 and st["evals"] == 1 + 6 * 3
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in log])
        e = maxrel(s.get_m(), o.m)
        note("512x512 dp45 variants", (rv, cv), "attempts", log, "m maxrel", e)
        assert e <= 1e-5


def test_block_kernels_256_periodic_rows(lib):
    """The 3D block's kernels at 256 x 64 x 64 cells: rows of 256 periodic
    cells (natural layout, the row pass of the 256 x 256 x 64 block), y
    periodic of 64 and z open of 128 (tiled column passes), 300 K thermal
    field: H_eff at a step and two Heun steps, against the oracle."""
    prob, m0, run = workloads.film_3d((256, 64, 64))
    prob["images"] = 1
    note("case: 256x64x64 periodic x/y, thermal, images 1")
    s = solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    s.step("heun", run["dt"], 1)
    o.step("heun", run["dt"], 1)
    m1 = s.get_m()
    e = maxrel(m1, o.m)
    note("  heun 1 step: m maxrel", e)
    assert e <= 1e-5
    h = s.eval_heff()
    ref = fields.heff(m1.astype(np.float64), prob, dt=run["dt"], step=1)
    eh = maxrel(h, ref)
    note("  H_eff (thermal draw of step 1): maxrel", eh)
    assert eh <= 1e-5
    s.step("heun", run["dt"], 1)
    o.step("heun", run["dt"], 1)
    e = maxrel(s.get_m(), o.m)
    note("  heun 2 steps: m maxrel", e)
    assert e <= 1e-5


@pytest.mark.parametrize("method", ["heun", "rk4"])
def test_periodic_256_rows_thermal_steps(lib, method):
    """Several fixed steps with the thermal field on rows of 256 periodic
    cells (256 x 32 x 4, periodic x and y), against the oracle."""
    prob, m0, run = workloads.film_3d((256, 32, 4))
    prob["images"] = 3
    note("case: 256x32x4 periodic x/y, thermal,", method)
    s = solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    for blk in range(2):
        s.step(method, run["dt"], 3)
        o.step(method, run["dt"], 3)
        e = maxrel(s.get_m(), o.m)
        note("  steps", 3 * (blk + 1), "m maxrel", e)
        assert e <= 1e-5


# ragged films of compiled padded lengths: 2 n is no 2,3,5,7-smooth length,
# so the padding goes to the next compiled one (127 -> 256, 31 -> 64, 191 ->
# 384, 95 -> 192, 383 -> 768, 509 -> 1024)
RAGGED = [(127, 31), (31, 127), (191, 95), (383, 95), (509, 31)]


@pytest.mark.parametrize("n", RAGGED, ids=lambda n: f"{n[0]}x{n[1]}")
def test_every_variant_ragged(lib, default_variants, n):
    """Every (row, column) variant pair on a ragged film: H_eff and five RK4
    steps (the fused stage pass) against the oracle."""
    prob, m0 = workloads.small_problem((n[0], n[1], 1), seed=n[0] + 3 * n[1], alpha=0.3)
    ref = fields.heff(m0.astype(np.float64), prob)
    o = ollg.Solver(prob, m0)
    o.step("rk4", 1e-13, 5)
    tried = 0
    for rv in range(2):
        for cv in range(2):
            s = lib.Solver(0)
            s.set_problem(prob)
            try:
                s.set_variants(rv, cv)
            except lib.LLGError as err:
                assert err.code == lib.LLG_E_ARG and (rv, cv) != (0, 0)
                note(n, (rv, cv), "refused")
                continue
            s.set_m(m0)
            eh = maxrel(s.eval_heff(), ref)
            s.step("rk4", 1e-13, 5)
            em = maxrel(s.get_m(), o.m)
            note(n, (rv, cv), "H_eff maxrel", eh, "rk4 m maxrel", em)
            assert eh <= 1e-5 and em <= 1e-5
            tried += 1
    assert tried >= 2


def test_ragged_dp45_each_row_variant(lib, default_variants):
    """The first-stage forward pass with the stage combination and the
    error pass (Dormand-Prince) on a ragged film, both row variants."""
    prob, m0 = workloads.small_problem((191, 95, 1), seed=5, alpha=0.3)
    for rv in range(2):
        s = lib.Solver(0)
        s.set_problem(prob)
        s.set_variants(rv, 0)
        s.set_m(m0)
        st = s.run(2e-12, 1e-5, 1e-14)
        assert st["done"] == 1
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in s.attempts()])
        e = maxrel(s.get_m(), o.m)
        note("191x95 dp45 row variant", rv, "attempts", len(s.attempts()), "m maxrel", e)
        assert e <= 1e-5


def test_two_solvers_keep_their_variants(lib, default_variants):
    """A solver keeps the variants it was set up with while another solver
    of the same lengths tunes or switches (and so changes the table of
    defaults): its captured steps and cached spectrum stay consistent, so it
    continues bit for bit like an undisturbed solver, and both follow the
    oracle."""
    prob, m0 = workloads.small_problem((64, 64, 1), seed=12, alpha=0.3)
    a = solver(lib, prob, m0)
    ref = solver(lib, prob, m0)
    for x in (a, ref):
        x.run(1e-12, 1e-5, 1e-14)
        x.step("rk4", 1e-13, 3)
    b = solver(lib, prob, m0)
    b.set_variants(1, 1)          # also the defaults for 128-point rows and 64-point columns
    b.run(1e-12, 1e-5, 1e-14)
    c = solver(lib, prob, m0)     # set up after the switch: variants (1, 1)
    for x in (a, ref):
        x.step("rk4", 1e-13, 3)
        x.run(3e-12, 1e-5, 0.0)
    assert np.array_equal(a.get_m(), ref.get_m())
    assert a.attempts() == ref.attempts()
    o = ollg.Solver(prob, m0)
    o.replay([(dt, ok) for dt, _, ok in b.attempts()])
    e = maxrel(b.get_m(), o.m)
    note("switched solver m maxrel", e)
    assert e <= 1e-5
    c.run(1e-12, 1e-5, 1e-14)
    assert np.array_equal(c.get_m(), b.get_m())
    b.autotune(2)
    a.step("rk4", 1e-13, 2)
    ref.step("rk4", 1e-13, 2)
    assert np.array_equal(a.get_m(), ref.get_m())


def test_eval_after_finished_run(lib):
    """An adaptive run that reached t_end leaves the device-side done flag
    set; H_eff evaluated afterwards is still that of the final state (equal
    bit for bit to a fresh solver's evaluation of the same m), and the run
    still reports itself done."""
    prob, m0 = workloads.small_problem((64, 32, 1), seed=4, alpha=0.3)
    s = solver(lib, prob, m0)
    st = s.run(1e-12, 1e-5, 1e-14)
    assert st["done"] == 1
    h = s.eval_heff()
    # the fresh solver takes the final state through set_state, which keeps
    # m bit for bit (set_m would renormalise it once more)
    fresh = lib.Solver(0)
    fresh.set_problem(prob)
    state, m_fin = s.get_state()
    fresh.set_state(state, m_fin)
    assert np.array_equal(fresh.get_m(), s.get_m())
    assert np.array_equal(h, fresh.eval_heff())
    assert s.stats()["done"] == 1
    ref = fields.heff(s.get_m().astype(np.float64), prob)
    assert maxrel(h, ref) <= 1e-5
