"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Error measures: max-relative = max_cells |v_gpu - v_ref| / max_cells |v_ref|
(vector norms per cell), RMS-relative = sqrt(sum |dv|^2 / sum |v_ref|^2).
The FP32 bar for H_eff is 1e-5 max-relative (single-precision FFTs with
FP64-rounded twiddles give ~1e-6; the product with the kernel and the
local terms add a few ulps)."""
import math
import sys

import numpy as np
import pytest

import workloads
from oracle import demag, fields, llg as ollg

pytestmark = pytest.mark.gpu


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(3, -1)
    b = np.asarray(b, dtype=np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


def rmsrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(math.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def note(*args):
    print(*args, flush=True)
    sys.stdout.flush()


@pytest.fixture(params=["fast", "generic"])
def impl(request, monkeypatch):
    """Runs a test with the compiled-length kernels (when the sizes allow)
    and again with the runtime-length kernels forced everywhere."""
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
# FFT (PIN-7)
# --------------------------------------------------------------------------
FFT_SIZES = [1, 2, 3, 4, 5, 7, 8, 12, 16, 20, 28, 32, 48, 64, 96, 128, 160, 192, 224, 256, 384,
             448, 512, 640, 768, 1024, 1536, 2048, 4096]


@pytest.mark.parametrize("n", FFT_SIZES)
def test_fft_matches_numpy_and_roundtrips(lib, n):
    note("fft", n)
    rng = np.random.default_rng(n)
    batch = max(1, min(64, 8192 // n))
    x = (rng.standard_normal((batch, n)) + 1j * rng.standard_normal((batch, n))).astype(np.complex64)
    s = lib.Solver(0)
    inv = s.fft_roundtrip(x.copy(), inverse_only=True)
    ref = np.fft.ifft(x.astype(np.complex128), axis=1)
    assert np.max(np.abs(inv - ref)) <= 2e-6 * np.max(np.abs(ref)) * max(1.0, math.log2(n))
    rt = s.fft_roundtrip(x.copy())
    err = np.max(np.abs(rt - x)) / np.max(np.abs(x))
    note("  roundtrip err", err)
    assert err < 5e-6          # the paper reports O(1e-6) at these sizes


# --------------------------------------------------------------------------
# demag tensor (FP64 on the GPU vs the oracle)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,pbc,cell", [((40, 30, 1), (False,) * 3, (4e-9, 4e-9, 3e-9)),
                                        ((16, 12, 10), (True, True, False), (3e-9, 3e-9, 3e-9)),
                                        ((9, 12, 6), (False, True, True), (2e-9, 3e-9, 2.5e-9))])
def test_demag_tensor_entries(lib, n, pbc, cell):
    note("tensor", n, pbc)
    rng = np.random.default_rng(1)
    offs = np.stack([rng.integers(-(n[a] - 1), n[a], 300) for a in range(3)], axis=1)
    offs[:20] = 0
    offs[1:20, 0] = np.arange(1, 20) % n[0]
    s = lib.Solver(0)
    s.set_geometry(n, pbc, images=3)
    s.set_cellsize(cell)
    got = s.demag_tensor(offs)
    geom = {"n": n, "cell": cell, "pbc": pbc, "images": 3}
    ref = demag.kernel_for_offsets(offs[:, 0], offs[:, 1], offs[:, 2], geom).T
    scale = np.abs(ref).max()
    assert np.max(np.abs(got - ref)) <= 1e-10 * scale


# --------------------------------------------------------------------------
# H_eff parity, per term and total
# --------------------------------------------------------------------------
CASES = [
    dict(n=(8, 6, 1)),
    dict(n=(17, 9, 1)),                                         # ragged, non-2^n padding
    dict(n=(32, 32, 1), cell=(4e-9, 4e-9, 4e-9)),
    dict(n=(70, 45, 1)),                                        # several column tiles, ragged
    dict(n=(6, 5, 4)),                                          # 3D open
    dict(n=(8, 8, 3), pbc=(True, True, False), cell=(3e-9, 3e-9, 3e-9)),
    dict(n=(12, 10, 5), pbc=(True, False, True)),
    dict(n=(16, 6, 2), pbc=(False, True, False)),
    dict(n=(64, 96, 1)),                                        # compiled 3*2^k column length
    dict(n=(96, 64, 1)),                                        # compiled 3*2^k row length
    dict(n=(128, 32, 1), pbc=(False, False, False)),
    dict(n=(64, 30, 1)),                                        # ragged rows below the padding
    # 3D with an open z axis of compiled half length (tiled z pass), ragged
    # kx tiles, periodic x/y with an odd y length, z shorter than the half
    dict(n=(12, 10, 16)),
    dict(n=(20, 9, 32), pbc=(True, True, False), cell=(3e-9, 3e-9, 3e-9)),
    dict(n=(6, 5, 64)),
    dict(n=(8, 6, 31)),
    dict(n=(5, 4, 128), cell=(3e-9, 3e-9, 3e-9)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c["n"])) + "-" +
                         "".join("p" if p else "o" for p in c.get("pbc", (False,) * 3)))
@pytest.mark.parametrize("term", ["demag", "exchange", "anisotropy", "zeeman", "all"])
def test_heff_parity(lib, impl, case, term):
    prob, m0 = workloads.small_problem(**case)
    if term != "all":
        prob["terms"] = (term,)
    note("heff", case, term)
    s = make_solver(lib, prob, m0)
    h = s.eval_heff()
    ref = fields.heff(m0.astype(np.float64), prob)
    e = maxrel(h, ref)
    note("  maxrel", e, "rmsrel", rmsrel(h, ref))
    assert e <= 1e-5


# 3D grids whose y or z axis has a compiled length (tiled column passes):
# open and periodic y of 32 ... 512, periodic z, ragged kx tiles
CASES_3D_TILED = [
    dict(n=(10, 16, 8)),
    dict(n=(8, 32, 16), pbc=(False, True, False)),
    dict(n=(6, 64, 6), pbc=(True, True, False), cell=(3e-9, 3e-9, 3e-9)),
    dict(n=(5, 64, 4)),
    dict(n=(4, 128, 4), pbc=(False, True, False)),
    dict(n=(3, 128, 3)),
    dict(n=(4, 256, 3), pbc=(False, True, False), cell=(3e-9, 3e-9, 3e-9)),
    dict(n=(3, 256, 2)),
    dict(n=(4, 6, 32), pbc=(False, False, True)),
    # compiled x lengths: the fast row kernels with the natural 3D layout
    dict(n=(32, 6, 4)),
    dict(n=(64, 5, 3), pbc=(True, False, False)),
    dict(n=(96, 4, 3)),
    dict(n=(64, 32, 16), pbc=(True, True, False), cell=(3e-9, 3e-9, 3e-9)),
]


@pytest.mark.parametrize("method", ["heun", "rk4"])
def test_3d_fast_rows_fixed_steps(lib, impl, method):
    """Fixed steps on a 3D grid whose rows have a compiled length (periodic
    x): the fused row pass with the next stage's forward transform in the
    natural layout, against the oracle over 20 steps."""
    prob, m0 = workloads.small_problem(n=(64, 6, 4), pbc=(True, False, False), alpha=0.5)
    s = make_solver(lib, prob, m0)
    s.step(method, 1e-13, 20)
    o = ollg.Solver(prob, m0)
    o.step(method, 1e-13, 20)
    e = maxrel(s.get_m(), o.m)
    note("3d fast rows", method, impl, "m maxrel", e)
    assert e <= 1e-5


def test_3d_fast_rows_dp45_replay(lib, impl):
    prob, m0 = workloads.small_problem(n=(32, 6, 4), alpha=0.5)
    s = make_solver(lib, prob, m0)
    st = s.run(3e-12, 1e-5, 1e-14)
    log = s.attempts()
    assert st["done"] == 1
    o = ollg.Solver(prob, m0)
    o.replay([(dt, ok) for dt, _, ok in log])
    e = maxrel(s.get_m(), o.m)
    note("3d fast rows dp45", impl, "attempts", len(log), "m maxrel", e)
    assert e <= 1e-5


@pytest.mark.parametrize("case", CASES_3D_TILED, ids=lambda c: "x".join(map(str, c["n"])) + "-" +
                         "".join("p" if p else "o" for p in c.get("pbc", (False,) * 3)))
@pytest.mark.parametrize("term", ["demag", "all"])
def test_heff_parity_3d_tiled(lib, impl, case, term):
    prob, m0 = workloads.small_problem(**case)
    if term != "all":
        prob["terms"] = (term,)
    note("heff 3d tiled", case, term)
    s = make_solver(lib, prob, m0)
    h = s.eval_heff()
    ref = fields.heff(m0.astype(np.float64), prob)
    e = maxrel(h, ref)
    note("  maxrel", e, "rmsrel", rmsrel(h, ref))
    assert e <= 1e-5


@pytest.mark.parametrize("case", [dict(n=(17, 9, 1)), dict(n=(64, 96, 1)), dict(n=(6, 5, 4)),
                                  dict(n=(8, 8, 3), pbc=(True, True, False), cell=(3e-9, 3e-9, 3e-9))],
                         ids=lambda c: "x".join(map(str, c["n"])))
@pytest.mark.parametrize("term", ["anisotropy", "all"])
def test_heff_parity_cubic(lib, impl, case, term):
    """Cubic anisotropy (Eq. 5) along rotated axes, with the uniaxial term."""
    prob, m0 = workloads.small_problem(**case)
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    prob.update(Kc1=4e4, Kc2=-2.5e4, c1=tuple(q[:, 0]), c2=tuple(q[:, 1]))
    if term != "all":
        prob["terms"] = (term,)
    s = make_solver(lib, prob, m0)
    h = s.eval_heff()
    ref = fields.heff(m0.astype(np.float64), prob)
    e = maxrel(h, ref)
    note("cubic", case, term, "maxrel", e)
    assert e <= 1e-5


@pytest.mark.parametrize("K1,kind", [(5e5, "100"), (-5e5, "111")])
def test_cubic_macrospin_on_gpu(lib, K1, kind):
    """A strongly damped single cell relaxes onto the nearest easy axis of
    the cubic term: the cube axes for K1 > 0, the body diagonals for K1 < 0."""
    rng = np.random.default_rng(11)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    c1, c2 = q[:, 0], q[:, 1]
    c3 = np.cross(c1, c2)
    easy = c1 if kind == "100" else (c1 + c2 + c3) / np.sqrt(3.0)
    perp = np.cross(easy, rng.standard_normal(3))
    perp /= np.linalg.norm(perp)
    m0 = (np.cos(0.4) * easy + np.sin(0.4) * perp).astype(np.float32).reshape(3, 1, 1, 1)
    prob = dict(n=(1, 1, 1), cell=(5e-9,) * 3, pbc=(False,) * 3, Ms=8e5, Aex=1.3e-11, alpha=1.0,
                Ku=0.0, Kc1=K1, Kc2=0.0, c1=tuple(c1), c2=tuple(c2), B=(0.0, 0.0, 0.0), T=0.0, seed=0)
    s = make_solver(lib, prob, m0)
    s.step("rk4", 1e-13, 3000)
    assert np.max(np.abs(s.get_m()[:, 0, 0, 0] - easy)) < 1e-5


def _stt_spiral(n, kc, alpha, xi, ny=1, along="x"):
    """In-plane spiral on a ring periodic along the current, field terms
    off: only the Zhang-Li torque acts."""
    dx = 3e-9
    q = 2 * np.pi * kc / (n * dx)
    th = q * np.arange(n) * dx
    if along == "x":
        m0 = np.stack([np.cos(th), np.sin(th), np.zeros(n)])[:, None, None, :].repeat(ny, axis=2)
        prob = dict(n=(n, ny, 1), pbc=(True, False, False), j=(1e12, 0.0, 0.0))
    else:
        m0 = np.stack([np.cos(th), np.sin(th), np.zeros(n)])[:, None, :, None].repeat(ny, axis=3)
        prob = dict(n=(ny, n, 1), pbc=(False, True, False), j=(0.0, 1e12, 0.0))
    prob.update(cell=(dx, dx, dx), Ms=8e5, Aex=1.3e-11, alpha=alpha, terms=(), P=0.6, xi=xi, T=0.0,
                seed=0, images=0)
    return prob, m0.astype(np.float32)


@pytest.mark.parametrize("along", ["x", "y"])
def test_stt_adiabatic_spiral_on_gpu(lib, impl, along):
    """Eq. 7 with xi = alpha and no field: the spiral turns rigidly; the GPU
    trajectory follows the oracle's (which is pinned to the closed form)."""
    # along x: 64 x 32 cells (compiled lengths, periodic rows); along y: 4 x 32
    prob, m0 = _stt_spiral(64 if along == "x" else 32, 2, 0.1, 0.1, ny=32 if along == "x" else 4, along=along)
    s = make_solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    s.step("rk4", 1e-13, 100)
    o.step("rk4", 1e-13, 100)
    e = maxrel(s.get_m(), o.m)
    note("stt adiabatic", along, e)
    assert e <= 1e-5


def test_stt_with_fields_parity(lib, impl):
    """The torque with every field term on, a non-adiabatic current at an
    angle and free edges (one-sided differences there): fixed steps against
    the oracle."""
    prob, m0 = workloads.small_problem(n=(64, 32, 1), alpha=0.3)
    prob.update(j=(8e11, -5e11, 0.0), P=0.7, xi=0.05)
    s = make_solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    for _ in range(3):
        s.step("rk4", 2e-14, 20)
        o.step("rk4", 2e-14, 20)
        e = maxrel(s.get_m(), o.m)
        note("stt fields", e)
        assert e <= 1e-5


def test_stt_uniform_state_on_gpu(lib):
    """A uniform state has no gradient: the current changes nothing."""
    prob, _ = workloads.small_problem(n=(16, 12, 1), alpha=0.2)
    m0 = workloads.uniform((16, 12, 1), (0.6, 0.0, 0.8))
    prob["terms"] = ()
    a = make_solver(lib, prob, m0)
    a.step("heun", 1e-13, 10)
    prob.update(j=(1e12, 3e11, 0.0), P=0.6, xi=0.05)
    b = make_solver(lib, prob, m0)
    b.step("heun", 1e-13, 10)
    assert np.array_equal(a.get_m(), b.get_m())


def test_heff_parity_film_32(lib, impl):
    prob, m0, _ = workloads.film_32()
    s = make_solver(lib, prob, m0)
    h = s.eval_heff()
    ref = fields.heff(m0.astype(np.float64), prob)
    e = maxrel(h, ref)
    note("film_32 heff maxrel", e, "rms", rmsrel(h, ref))
    assert e <= 1e-5


def test_heff_parity_film_512(lib, impl):
    """The full 512 x 512 film the benchmark times, every output compared."""
    prob, m0, _ = workloads.film_512()
    m0 = workloads.random_unit(prob["n"], 11)   # a rich state exercises every frequency
    s = make_solver(lib, prob, m0)
    h = s.eval_heff()
    ref = fields.heff(m0.astype(np.float64), prob)
    e = maxrel(h, ref)
    note("film_512 heff maxrel", e, "rms", rmsrel(h, ref))
    assert e <= 1e-5


def test_macrospin_cell(lib):
    """One cubic cell (the smallest FFT grid): self-demag -Ms/3 m plus B/mu0."""
    prob = dict(n=(1, 1, 1), cell=(5e-9,) * 3, pbc=(False,) * 3, Ms=8e5, Aex=1.3e-11, alpha=0.1,
                Ku=0.0, u=(1, 0, 0), B=(0.0, 0.0, 0.1), T=0.0, seed=0)
    m0 = workloads.uniform((1, 1, 1), (0.3, 0.4, 0.866))
    s = make_solver(lib, prob, m0)
    h = s.eval_heff()
    ref = fields.heff(m0.astype(np.float64), prob)
    assert maxrel(h, ref) <= 1e-6


# --------------------------------------------------------------------------
# trajectories
# --------------------------------------------------------------------------
@pytest.mark.parametrize("method", ["euler", "heun", "rk3", "rk4"])
def test_fixed_step_parity_small(lib, impl, method):
    prob, m0 = workloads.small_problem(n=(32, 32, 1), alpha=0.3)
    s = make_solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    for _ in range(4):
        s.step(method, 2e-14, 25)
        o.step(method, 2e-14, 25)
        e = maxrel(s.get_m(), o.m)
        note(method, "m maxrel", e)
        assert e <= 1e-5
    st = s.stats()
    assert st["steps"] == 100
    assert st["t"] == pytest.approx(100 * 2e-14, rel=1e-12)


@pytest.mark.parametrize("method", ["heun", "rk4"])
def test_film_32_trajectory(lib, impl, method):
    """1000 fixed steps at dt = 1e-13 s from a random state, m and H_eff
    compared every 100 steps (the strong damping keeps this comparison well
    conditioned: a 1e-7 nudge of the start state moves the oracle's m by
    about 5e-6)."""
    prob, m0, run = workloads.film_32()
    s = make_solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    worst_m, worst_h = 0.0, 0.0
    for blk in range(run["steps"] // 100):
        s.step(method, run["dt"], 100)
        o.step(method, run["dt"], 100)
        mg = s.get_m()
        em = maxrel(mg, o.m)
        # field parity on the same state (the GPU's): the trajectories'
        # own drift is measured by em
        eh = maxrel(s.eval_heff(), fields.heff(mg.astype(np.float64), prob))
        worst_m, worst_h = max(worst_m, em), max(worst_h, eh)
        note(method, (blk + 1) * 100, "m maxrel", em, "H maxrel", eh)
    assert worst_m <= 1e-5
    assert worst_h <= 1e-5


def oracle_sensitivity(prob, m0, attempts, seed=0, method="rkdp45"):
    """How far the FP64 oracle itself moves when its start state is nudged
    by 3e-8 per component (FP32 rounding size) and replayed along the same
    attempts: the
    conditioning of the comparison.  A parity bar of 1e-5 is only
    meaningful where this stays well below it."""
    rng = np.random.default_rng(seed)
    a = ollg.Solver(prob, m0)
    a.replay(attempts, method)
    b = ollg.Solver(prob, m0.astype(np.float64) + 3e-8 * rng.standard_normal(m0.shape))
    b.replay(attempts, method)
    return maxrel(b.m, a.m)


@pytest.mark.parametrize("name,prob_m,t_end", [
    ("random-24x20-a0.5", lambda: workloads.small_problem(n=(24, 20, 1), alpha=0.5), 5e-12),
    ("film_512-scaled-64", lambda: workloads.film_512(64)[:2], 2e-11),
])
def test_dp45_replay_parity(lib, impl, name, prob_m, t_end):
    """Adaptive Dormand-Prince on the GPU; the oracle replays the GPU's
    recorded step sizes and acceptances (the exact dt sequence depends on
    rounding), then m is compared, and the oracle's own error estimates
    agree with the GPU's."""
    prob, m0 = prob_m()
    s = make_solver(lib, prob, m0)
    st = s.run(t_end, 1e-5, 1e-14)
    log = s.attempts()
    note(name, "dp45 stats", st, "attempts", len(log))
    assert st["done"] == 1 and st["t"] == pytest.approx(t_end, rel=1e-12)
    assert len(log) == st["steps"] + st["rejected"]
    attempts = [(dt, ok) for dt, _, ok in log]
    sens = oracle_sensitivity(prob, m0, attempts)
    o = ollg.Solver(prob, m0)
    errs = o.replay(attempts)
    e = maxrel(s.get_m(), o.m)
    note(name, "dp45 m maxrel", e, "oracle sensitivity", sens)
    assert sens <= 2e-6
    assert e <= 1e-5
    for (dt, eg, ok), eo in zip(log, errs):
        assert eg == pytest.approx(eo, rel=2e-2, abs=1e-8)


@pytest.mark.parametrize("method", ["rk23", "rkck", "rk12"])
def test_embedded_pair_replay_parity(lib, impl, method):
    """The other adaptive pairs of Sec. 2.2 on the GPU, replayed by the
    oracle along the GPU's step sizes and acceptances: m to 1e-5 and every
    attempt's error estimate to 2e-2."""
    prob, m0 = workloads.small_problem(n=(24, 20, 1), alpha=0.5)
    t_end = 5e-12
    s = make_solver(lib, prob, m0)
    st = s.run(t_end, 1e-5, 1e-14, method=method)
    log = s.attempts()
    note(method, "stats", st, "attempts", len(log))
    assert st["done"] == 1 and st["t"] == pytest.approx(t_end, rel=1e-12)
    assert len(log) == st["steps"] + st["rejected"]
    attempts = [(dt, ok) for dt, _, ok in log]
    sens = oracle_sensitivity(prob, m0, attempts, method=method)
    o = ollg.Solver(prob, m0)
    errs = o.replay(attempts, method)
    e = maxrel(s.get_m(), o.m)
    note(method, "m maxrel", e, "oracle sensitivity", sens)
    assert sens <= 2e-6
    assert e <= 1e-5
    for (dt, eg, ok), eo in zip(log, errs):
        assert eg == pytest.approx(eo, rel=2e-2, abs=1e-8)
    # the step sizes follow the pair's controller: after each attempt the
    # next one is dt * clamp(0.9 (tol/err)^(1/(q+1)), 0.2, 5), or the rest
    q = ollg.ADAPTIVE[method][1]
    t = 0.0
    for (dt, eg, ok), (dn, _, _) in zip(log[:-1], log[1:]):
        t = t + dt if ok else t
        want = ollg.Solver.next_dt(dt, eg, 1e-5, q)
        assert dn == pytest.approx(min(want, t_end - t), rel=1e-6)
    # evaluations per attempt: S - 1 with first-same-as-last, else S (and
    # one start-up evaluation for the former)
    tab, _ = ollg.ADAPTIVE[method]
    S = len(tab["b"])
    fsal = method == "rk23"
    assert st["evals"] == len(log) * (S - 1 if fsal else S) + (1 if fsal else 0)


def test_dp45_film_512_scaled_reanchored(lib, impl):
    """Longer adaptive run (100 ps, 64 x 64 version of the benchmark film):
    the dynamics amplify rounding, so the oracle restarts from the GPU's
    state at every 10 ps checkpoint and must reproduce the GPU's next
    segment, replaying its attempts, to 1e-5."""
    prob, m0, run = workloads.film_512(64)
    s = make_solver(lib, prob, m0)
    t, worst, seen = 0.0, 0.0, 0
    m_start = m0
    for seg in range(10):
        t += 1e-11
        s.run(t, run["tol"], run["dt0"] if seg == 0 else s.stats()["dt_next"])
        log = s.attempts()
        chunk = [(dt, ok) for dt, _, ok in log[seen:]]
        seen = len(log)
        o = ollg.Solver(prob, m_start)
        o.replay(chunk)
        m_gpu = s.get_m()
        e = maxrel(m_gpu, o.m)
        worst = max(worst, e)
        note("segment", seg, "attempts", len(chunk), "m maxrel", e)
        m_start = m_gpu
    assert worst <= 1e-5


def test_macrospin_precession_on_gpu(lib):
    """PIN-11 on the GPU path: one cube cell precesses and damps as the
    closed form says."""
    alpha, Bz = 0.1, 0.1
    th0, ph0 = 1.0, 0.3
    prob = dict(n=(1, 1, 1), cell=(5e-9,) * 3, pbc=(False,) * 3, Ms=8e5, Aex=1.3e-11, alpha=alpha,
                Ku=0.0, u=(1, 0, 0), B=(0.0, 0.0, Bz), T=0.0, seed=0)
    m0 = np.array([math.sin(th0) * math.cos(ph0), math.sin(th0) * math.sin(ph0), math.cos(th0)],
                  dtype=np.float32).reshape(3, 1, 1, 1)
    s = make_solver(lib, prob, m0)
    s.step("rk4", 1e-13, 2000)
    H = Bz / (4e-7 * math.pi)
    w = 4e-7 * math.pi * 1.7595e11 * H / (1 + alpha ** 2)
    t = 2e-10
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * w * t))
    ph = ph0 + w * t
    exact = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    assert np.max(np.abs(s.get_m()[:, 0, 0, 0] - exact)) < 2e-5


# --------------------------------------------------------------------------
# errors
# --------------------------------------------------------------------------
def test_error_paths(lib):
    s = lib.Solver(0)
    with pytest.raises(lib.LLGError) as e:
        s.eval_heff()
    assert e.value.code in (lib.LLG_E_STATE, lib.LLG_E_ARG)
    prob, m0 = workloads.small_problem()
    s.set_problem(prob)
    with pytest.raises(lib.LLGError) as e:
        s.eval_heff()
    assert e.value.code == lib.LLG_E_STATE
    bad = m0.copy()
    bad[0, 0, 0, 0] *= 1.1
    with pytest.raises(lib.LLGError) as e:
        s.set_m(bad)
    assert e.value.code == lib.LLG_E_ARG
    with pytest.raises(lib.LLGError) as e:
        s.set_material(-1.0, 1e-11, 0.1)
    assert e.value.code == lib.LLG_E_ARG
    with pytest.raises(lib.LLGError) as e:
        s.set_geometry((7, 5, 1), (True, False, False))
    assert e.value.code == lib.LLG_E_UNSUPPORTED


# --------------------------------------------------------------------------
# thermal field and the 3D periodic path
# --------------------------------------------------------------------------
def test_thermal_steps_parity(lib):
    """Fixed Heun steps with only the applied and thermal fields: the GPU
    and the oracle draw the same Philox stream (24-bit uniforms, Box-Muller
    in each precision), so the trajectories agree to rounding."""
    prob, m0 = workloads.small_problem(n=(16, 12, 1), T=300.0, seed=77,
                                       terms=("zeeman", "thermal"), alpha=0.1)
    dt = 5e-14
    s = make_solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    s.step("heun", dt, 10)
    o.step("heun", dt, 10)
    e = maxrel(s.get_m(), o.m)
    note("thermal heun m maxrel", e)
    assert e <= 1e-5
    h = s.eval_heff()
    ref = fields.heff(s.get_m().astype(np.float64), prob, dt=dt, step=10)
    eh = maxrel(h, ref)
    note("thermal field maxrel", eh)
    assert eh <= 1e-5


def test_film_3d_scaled_parity(lib):
    """The 3D workload's physics at 16 x 16 x 8 cells: periodic in x and y,
    open z, 300 K thermal field, vortex start, Heun at 5e-14 s."""
    prob, m0, run = workloads.film_3d((16, 16, 8))
    prob["images"] = 3
    s = make_solver(lib, prob, m0)
    o = ollg.Solver(prob, m0)
    for blk in range(3):
        s.step("heun", run["dt"], 5)
        o.step("heun", run["dt"], 5)
        e = maxrel(s.get_m(), o.m)
        note("3d step", (blk + 1) * 5, "m maxrel", e)
        assert e <= 1e-5


def test_film_3d_heff_parity(lib):
    prob, m0, run = workloads.film_3d((32, 16, 6))
    prob["images"] = 4
    prob["terms"] = ("demag", "exchange", "anisotropy", "zeeman")
    s = make_solver(lib, prob, m0)
    h = s.eval_heff()
    ref = fields.heff(m0.astype(np.float64), prob)
    e = maxrel(h, ref)
    note("3d heff maxrel", e)
    assert e <= 1e-5
