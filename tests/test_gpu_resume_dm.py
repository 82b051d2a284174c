"""The fixed-tableau integrators with a bounded variation of m per step
(Sec. 2.2) and checkpoint/resume through the C ABI, against the FP64 oracle
and against uninterrupted runs of the library itself."""
import math
import sys

import numpy as np
import pytest

import workloads
from oracle import llg as ollg
from oracle.constants import GAMMA0, MU0

pytestmark = pytest.mark.gpu


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(3, -1)
    b = np.asarray(b, dtype=np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


def note(*args):
    print(*args, flush=True)
    sys.stdout.flush()


@pytest.fixture(params=["fast", "generic"])
def impl(request, monkeypatch):
    if request.param == "generic":
        monkeypatch.setenv("LLG_FORCE_GENERIC", "1")
    else:
        monkeypatch.delenv("LLG_FORCE_GENERIC", raising=False)
    return request.param


def make_solver(lib, prob, m0):
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    return s


# --------------------------------------------------------------------------
# bounded variation of m per step
# --------------------------------------------------------------------------
@pytest.mark.parametrize("method", ["euler", "heun", "rk3", "rk4"])
def test_dm_run_replay_parity(lib, impl, method):
    """The GPU picks every step on the device; the oracle takes the same
    steps and must land on the same m (1e-5), and its own choice of each step
    (from its FP64 max |dm/dt|) must agree with the GPU's."""
    prob, m0 = workloads.small_problem(n=(24, 20, 1), alpha=0.5)
    t_end, max_dm, dt_max = 2e-12, 1e-2, 1e-12
    s = make_solver(lib, prob, m0)
    st = s.run_dm(method, t_end, max_dm, dt_max)
    log = s.attempts()
    note(method, impl, "stats", st, "steps", len(log))
    assert st["done"] == 1 and st["t"] == t_end
    S = len(ollg.TABLEAUX[method]["b"])
    assert st["steps"] == len(log) and st["rejected"] == 0 and st["evals"] == S * len(log)
    assert all(ok for _, _, ok in log)
    o = ollg.Solver(prob, m0)
    rec = o.run_dm(method, t_end, max_dm, dt_max, dts=[dt for dt, _, _ in log])
    e = maxrel(s.get_m(), o.m)
    note(method, impl, "m maxrel", e)
    assert e <= 1e-5
    for (dt, own), (_, err, _) in zip(rec[:-1], log[:-1]):
        assert dt == pytest.approx(own, rel=1e-4)
        # the recorded bound is max_dm unless dt_max capped the step
        if dt < dt_max * (1 - 1e-6):
            assert err == pytest.approx(max_dm, rel=1e-5)
    assert sum(dt for dt, _ in rec) == pytest.approx(t_end, rel=1e-12)


def test_dm_run_macrospin_on_gpu(lib):
    """Undamped macrospin: every step is max_dm / (gamma0 H sin theta0) and
    RK4 along them follows the closed-form precession."""
    Bz, th0, ph0 = 0.1, 1.0, 0.3
    prob = dict(n=(1, 1, 1), cell=(5e-9,) * 3, pbc=(False,) * 3, Ms=8e5, Aex=1.3e-11, alpha=0.0,
                Ku=0.0, u=(1, 0, 0), B=(0.0, 0.0, Bz), T=0.0, seed=0)
    m0 = np.array([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)],
                  dtype=np.float32).reshape(3, 1, 1, 1)
    s = make_solver(lib, prob, m0)
    t_end, max_dm = 2e-10, 1e-2
    st = s.run_dm("rk4", t_end, max_dm, 1e-9)
    log = s.attempts()
    h = max_dm / (GAMMA0 * Bz / MU0 * math.sin(th0))
    note("macrospin dm steps", len(log), "h", h, "first", log[0][0])
    assert st["t"] == t_end and len(log) == math.ceil(t_end / h)
    for dt, _, _ in log[:-1]:
        assert dt == pytest.approx(h, rel=1e-4)
    w = GAMMA0 * Bz / MU0
    exact = np.array([math.sin(th0) * math.cos(ph0 + w * t_end), math.sin(th0) * math.sin(ph0 + w * t_end),
                      math.cos(th0)])
    assert np.max(np.abs(s.get_m()[:, 0, 0, 0] - exact)) < 5e-5


def test_dm_run_rejects_bad_arguments(lib):
    prob, m0 = workloads.small_problem(n=(8, 8, 1))
    s = make_solver(lib, prob, m0)
    for args in [("rkdp45", 1e-12, 1e-2, 1e-13), ("rk4", 1e-12, 0.0, 1e-13), ("rk4", 1e-12, 1e-2, -1.0)]:
        with pytest.raises(lib.LLGError) as ei:
            s.run_dm(*args)
        assert ei.value.code == lib.LLG_E_ARG


# --------------------------------------------------------------------------
# checkpoint and resume
# --------------------------------------------------------------------------
def test_resume_fixed_thermal_steps_bitwise(lib):
    """Heun with the thermal field: 10 + 10 steps through a saved state in a
    fresh solver equal 20 steps in one solver, bit for bit (the Philox draw
    counter is part of the state)."""
    prob, m0 = workloads.small_problem(n=(32, 16, 1), alpha=0.1)
    prob = dict(prob, T=300.0, seed=11)
    a = make_solver(lib, prob, m0)
    a.step("heun", 1e-13, 20)
    b = make_solver(lib, prob, m0)
    b.step("heun", 1e-13, 10)
    state, m = b.get_state()
    note("state after 10 steps", state)
    assert state["step"] == 10 and state["t"] == pytest.approx(1e-12, rel=1e-12)
    c = lib.Solver(0)
    c.set_problem(prob)
    c.set_state(state, m)
    c.step("heun", 1e-13, 10)
    assert np.array_equal(c.get_m(), a.get_m())
    sa, sc = a.stats(), c.stats()
    for k in ("t", "steps", "evals"):
        assert sc[k] == sa[k], k


def test_resume_adaptive_run_bitwise(lib):
    """Dormand-Prince stopped after 15 attempts, saved, restored into a fresh
    solver and continued with dt0 = 0 (the controller's own next step) takes
    the same attempts as the uninterrupted run: same m bit for bit, same
    counts, except the one evaluation of f(m) the resumed first-same-as-last
    pair needs before its first attempt."""
    prob, m0 = workloads.small_problem(n=(24, 20, 1), alpha=0.5)
    t_end = 5e-12
    a = make_solver(lib, prob, m0)
    sa = a.run(t_end, 1e-5, 1e-14)
    b = make_solver(lib, prob, m0)
    b.run_attempts(t_end, 1e-5, 1e-14, 15)
    state, m = b.get_state()
    note("uninterrupted", sa, "state after 15 attempts", state)
    assert state["t"] < t_end and state["dt_next"] > 0
    c = lib.Solver(0)
    c.set_problem(prob)
    c.set_state(state, m)
    sc = c.run(t_end, 1e-5, 0.0)
    note("resumed", sc)
    assert np.array_equal(c.get_m(), a.get_m())
    for k in ("t", "dt", "dt_next", "max_err", "steps", "rejected"):
        assert sc[k] == sa[k], k
    assert sc["evals"] == sa["evals"] + 1


def test_resume_dm_run_bitwise(lib):
    """A run with bounded variation of m to t1, saved and restored into a
    fresh solver, then continued to t2, equals continuing in the first
    solver."""
    prob, m0 = workloads.small_problem(n=(24, 20, 1), alpha=0.5)
    a = make_solver(lib, prob, m0)
    a.run_dm("rk4", 1e-12, 1e-2, 1e-12)
    state, m = a.get_state()
    a.run_dm("rk4", 3e-12, 1e-2, 1e-12)
    c = lib.Solver(0)
    c.set_problem(prob)
    c.set_state(state, m)
    c.run_dm("rk4", 3e-12, 1e-2, 1e-12)
    assert np.array_equal(c.get_m(), a.get_m())
    assert c.stats()["steps"] == a.stats()["steps"]


def test_set_state_rejects_bad_records(lib):
    prob, m0 = workloads.small_problem(n=(8, 8, 1))
    s = make_solver(lib, prob, m0)
    s.step("rk4", 1e-13, 2)
    state, m = s.get_state()
    c = lib.Solver(0)
    c.set_problem(prob)
    for bad_state, bad_m in [(dict(state, health=1), m), (dict(state, steps=-1), m),
                             (dict(state, t=float("nan")), m), (state, 2.0 * m)]:
        with pytest.raises(lib.LLGError) as ei:
            c.set_state(bad_state, bad_m)
        assert ei.value.code == lib.LLG_E_ARG
    with pytest.raises(lib.LLGError) as ei:
        c.run(1e-12, 1e-5, 0.0)      # no state: dt0 = 0 has nothing to continue
    assert ei.value.code in (lib.LLG_E_STATE,)
    c.set_state(state, m)
    assert np.array_equal(c.get_m(), m)
