"""Pins of the oracle's field terms, thermal draw, LL right-hand side and
integrators against closed forms, invariants and order conditions (CPU)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import fields, llg, philox
from oracle.constants import MU0, GAMMA0, KB
import workloads


# --------------------------------------------------------------------------
# exchange (Eq. 3)
# --------------------------------------------------------------------------
def test_exchange_on_periodic_spiral_is_exact():
    """PIN-8: on a periodic spiral m = (cos kx, sin kx, 0) the six-neighbour
    Laplacian is exactly -(2 - 2 cos k d)/d^2 m."""
    nx, d = 24, 3e-9
    q = 5
    k = 2 * math.pi * q / (nx * d)
    x = (np.arange(nx) + 0.5) * d
    m = np.zeros((3, 2, 3, nx))
    m[0] = np.cos(k * x)
    m[1] = np.sin(k * x)
    prob = dict(n=(nx, 3, 2), cell=(d, 2e-9, 5e-9), pbc=(True, False, False),
                Ms=8e5, Aex=1.3e-11)
    H = fields.exchange_field(m, prob)
    expect = -2 * 1.3e-11 / (MU0 * 8e5) * (2 - 2 * math.cos(k * d)) / d ** 2 * m
    np.testing.assert_allclose(H, expect, atol=1e-9 * np.abs(expect).max())


def test_exchange_of_uniform_state_is_zero():
    prob, _ = workloads.small_problem(n=(5, 4, 3), pbc=(False, True, False))
    m = workloads.uniform((5, 4, 3), (0.3, -0.2, 0.9)).astype(np.float64)
    assert np.abs(fields.exchange_field(m, prob)).max() == 0.0


def test_exchange_free_edge_omits_missing_neighbour():
    """A two-cell chain: each cell has exactly one neighbour."""
    prob = dict(n=(2, 1, 1), cell=(2e-9, 2e-9, 2e-9), pbc=(False,) * 3, Ms=1e6, Aex=1e-11)
    m = np.zeros((3, 1, 1, 2))
    m[0, 0, 0, 0] = 1.0
    m[1, 0, 0, 1] = 1.0
    H = fields.exchange_field(m, prob)
    c = 2e-11 / (MU0 * 1e6) / 4e-18
    np.testing.assert_allclose(H[:, 0, 0, 0], c * (m[:, 0, 0, 1] - m[:, 0, 0, 0]))
    np.testing.assert_allclose(H[:, 0, 0, 1], c * (m[:, 0, 0, 0] - m[:, 0, 0, 1]))


# --------------------------------------------------------------------------
# energy consistency of every term
# --------------------------------------------------------------------------
@pytest.mark.parametrize("term", ["demag", "exchange", "anisotropy", "cubic", "zeeman"])
def test_field_is_minus_energy_gradient(term):
    """PIN-9: H = -(1/(mu0 Ms V)) dE/dm for each term, by central differences
    of the FP64 energy."""
    prob, m0 = workloads.small_problem(n=(4, 3, 2), pbc=(True, False, False), images=1)
    prob = dict(prob, Kc1=4e4, Kc2=-2e4, c1=(1.0, 1.0, 0.0), c2=(-1.0, 1.0, 0.5))
    if term == "cubic":
        prob["terms"] = ("anisotropy",)
        prob["Ku"] = 0.0
    elif term == "anisotropy":
        prob["terms"] = ("anisotropy",)
        prob["Kc1"] = prob["Kc2"] = 0.0
    else:
        prob["terms"] = (term,)
    m = m0.astype(np.float64)
    H = fields.heff(m, prob)
    dx, dy, dz = prob["cell"]
    V = dx * dy * dz
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(12):
        c = int(rng.integers(3))
        idx = tuple(int(rng.integers(s)) for s in m.shape[1:])
        mp = m.copy(); mp[(c,) + idx] += h
        mm = m.copy(); mm[(c,) + idx] -= h
        g = (fields.energy(mp, prob) - fields.energy(mm, prob)) / (2 * h)
        expect = -g / (MU0 * prob["Ms"] * V)
        assert H[(c,) + idx] == pytest.approx(expect, rel=1e-5, abs=1e-6 * np.abs(H).max())


# --------------------------------------------------------------------------
# thermal field (Eq. 6)
# --------------------------------------------------------------------------
KAT = [  # Philox4x32-10 known-answer vectors published with the generator
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    got = philox.philox4x32_10([np.array([c], dtype=np.uint32) for c in ctr], key)
    assert tuple(int(g[0]) for g in got) == out


def test_thermal_eta_moments():
    """PIN-14a: eta has mean 0, variance 1 and no correlation between
    neighbouring cells or consecutive steps."""
    n = 200000
    e0 = philox.thermal_eta(n, 0, 12345)
    e1 = philox.thermal_eta(n, 1, 12345)
    for e in (e0, e1):
        assert np.abs(e.mean(axis=1)).max() < 5 * 1 / math.sqrt(n)
        assert np.abs(e.var(axis=1) - 1).max() < 5 * math.sqrt(2 / n)
    lag_t = (e0 * e1).mean(axis=1)
    lag_x = (e0[:, 1:] * e0[:, :-1]).mean(axis=1)
    cross = (e0[0] * e0[1]).mean(), (e0[0] * e0[2]).mean()
    for v in list(lag_t) + list(lag_x) + list(cross):
        assert abs(v) < 5 / math.sqrt(n)


def test_thermal_sigma_value():
    prob, _, _ = workloads.film_3d()
    s = fields.thermal_sigma(prob, 5e-14)
    expect = math.sqrt(2 * 0.1 * KB * 300 / (GAMMA0 * MU0 * 1e6 * 27e-27 * 5e-14))
    assert s == pytest.approx(expect, rel=1e-14)
    assert s / 1e6 == pytest.approx(1.486, abs=1e-3)


@pytest.mark.slow
def test_langevin_equilibrium_of_independent_macrospins():
    """PIN-14b: an ensemble of uncoupled cube spins in a field B at
    temperature T relaxes to <cos theta> = coth(xi) - 1/xi with
    xi = mu0 Ms V H/(k_B T)."""
    n = (64, 64, 1)
    d = 5e-9
    Ms, T = 8e5, 300.0
    xi = 2.0
    H = xi * KB * T / (MU0 * Ms * d ** 3)
    prob = dict(n=n, cell=(d, d, d), pbc=(False,) * 3, Ms=Ms, Aex=0.0, alpha=0.5,
                B=(0.0, 0.0, MU0 * H), T=T, seed=99, terms=("zeeman", "thermal"))
    s = llg.Solver(prob, workloads.uniform(n, (0, 0, 1)))
    samples = []
    for block in range(30):
        s.step("heun", 1e-12, 50)
        if block >= 10:
            samples.append(float(s.m[2].mean()))
    mean = float(np.mean(samples))
    expect = 1 / math.tanh(xi) - 1 / xi
    assert mean == pytest.approx(expect, abs=0.015)


# --------------------------------------------------------------------------
# LL right-hand side (Eq. 1) and integrators (Sec. 2.2)
# --------------------------------------------------------------------------
def test_torque_is_orthogonal_to_m():
    """PIN-10a: m . f(m) = 0 for any field."""
    rng = np.random.default_rng(2)
    m = rng.standard_normal((3, 50))
    m /= np.linalg.norm(m, axis=0)
    H = rng.standard_normal((3, 50)) * 1e5
    f = llg.ll_rhs(m, H, 0.3)
    assert np.abs((m * f).sum(axis=0)).max() < 1e-9 * np.abs(f).max()


def _macrospin(alpha, Bz, theta0=1.0, phi0=0.3):
    """One cubic cell: its self-demag field is parallel to m, so only the
    applied field exerts a torque."""
    prob = dict(n=(1, 1, 1), cell=(5e-9,) * 3, pbc=(False,) * 3, Ms=8e5, Aex=1.3e-11,
                alpha=alpha, Ku=0.0, B=(0.0, 0.0, Bz), T=0.0, seed=0)
    m0 = np.array([math.sin(theta0) * math.cos(phi0), math.sin(theta0) * math.sin(phi0),
                   math.cos(theta0)]).reshape(3, 1, 1, 1)
    return prob, m0


def _macrospin_exact(alpha, Bz, t, theta0=1.0, phi0=0.3):
    H = Bz / MU0
    w = GAMMA0 * H / (1 + alpha * alpha)
    th = 2 * math.atan(math.tan(theta0 / 2) * math.exp(-alpha * w * t))
    ph = phi0 + w * t
    return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


def test_macrospin_closed_form():
    """PIN-11: precession at gamma0 H/(1+alpha^2) and damping of
    tan(theta/2) at rate alpha gamma0 H/(1+alpha^2), via the whole field
    pipeline (demag included)."""
    alpha, Bz = 0.1, 0.1
    prob, m0 = _macrospin(alpha, Bz)
    s = llg.Solver(prob, m0)
    s.step("rk4", 1e-13, 2000)
    np.testing.assert_allclose(s.m[:, 0, 0, 0], _macrospin_exact(alpha, Bz, 2e-10), atol=1e-9)


@pytest.mark.parametrize("method,order", [("euler", 1), ("heun", 2), ("rk3", 3), ("rk4", 4), ("rkdp45", 5),
                                          ("rk12", 2), ("rk23", 3), ("rkck", 5)])
def test_convergence_order(method, order):
    """PIN-12a: the global error on the macrospin problem falls as dt^p
    (embedded pairs: the order of the propagated solution)."""
    alpha, Bz, t_end = 0.2, 0.2, 1e-10
    errs = []
    # the fifth-order pairs reach their asymptotic rate only below ~1e-10 error here
    nsteps = (80, 160) if order == 5 else (40, 80)
    for n in nsteps:
        prob, m0 = _macrospin(alpha, Bz)
        s = llg.Solver(prob, m0)
        dt = t_end / n
        if method in llg.ADAPTIVE:
            for _ in range(n):
                s.m, _err = s.attempt(dt, method)
        else:
            s.step(method, dt, n)
        errs.append(np.abs(s.m[:, 0, 0, 0] - _macrospin_exact(alpha, Bz, t_end)).max())
    p = math.log2(errs[0] / errs[1])
    assert abs(p - order) < 0.35, (errs, p)


def _order_conditions(A, b, p):
    """The Butcher order conditions up to order p (all rooted trees up to
    order 5), with exact rational arithmetic."""
    s = len(b)
    A = [[Fraction(A[i][j]) if j < len(A[i]) else Fraction(0) for j in range(s)] for i in range(s)]
    b = [Fraction(x) for x in b]
    c = [sum(row) for row in A]
    dot = lambda u, v: sum(x * y for x, y in zip(u, v))
    Av = lambda v: [dot(row, v) for row in A]
    mul = lambda u, v: [x * y for x, y in zip(u, v)]
    one = [Fraction(1)] * s
    conds = [(dot(b, one), Fraction(1))]
    if p >= 2:
        conds += [(dot(b, c), Fraction(1, 2))]
    if p >= 3:
        conds += [(dot(b, mul(c, c)), Fraction(1, 3)), (dot(b, Av(c)), Fraction(1, 6))]
    if p >= 4:
        c2 = mul(c, c)
        conds += [(dot(b, mul(c2, c)), Fraction(1, 4)), (dot(b, mul(c, Av(c))), Fraction(1, 8)),
                  (dot(b, Av(c2)), Fraction(1, 12)), (dot(b, Av(Av(c))), Fraction(1, 24))]
    if p >= 5:
        c2 = mul(c, c)
        c3 = mul(c2, c)
        Ac = Av(c)
        conds += [(dot(b, mul(c3, c)), Fraction(1, 5)), (dot(b, mul(c2, Ac)), Fraction(1, 10)),
                  (dot(b, mul(c, Av(c2))), Fraction(1, 15)), (dot(b, mul(c, Av(Ac))), Fraction(1, 30)),
                  (dot(b, mul(Ac, Ac)), Fraction(1, 20)), (dot(b, Av(c3)), Fraction(1, 20)),
                  (dot(b, Av(mul(c, Ac))), Fraction(1, 40)), (dot(b, Av(Av(c2))), Fraction(1, 60)),
                  (dot(b, Av(Av(Ac))), Fraction(1, 120))]
    return conds


def _as_fractions(tab):
    # recover the exact rationals the tableaux were typed from
    conv = lambda x: Fraction(x).limit_denominator(10 ** 7)
    return [[conv(a) for a in row] for row in tab["A"]], [conv(x) for x in tab["b"]]


@pytest.mark.parametrize("name,p", [("euler", 1), ("heun", 2), ("rk3", 3), ("rk4", 4), ("rkdp45", 5),
                                    ("rk12", 2), ("rk23", 3), ("rkck", 5)])
def test_tableau_order_conditions(name, p):
    """PIN-12b: each tableau satisfies every order condition up to its
    order (a single mistyped coefficient fails one of them)."""
    A, b = _as_fractions(llg.TABLEAUX[name])
    for got, want in _order_conditions(A, b, p):
        assert got == want


def test_dp45_embedded_pair_is_fourth_order():
    A, _ = _as_fractions(llg.DP45)
    bh = [Fraction(x).limit_denominator(10 ** 7) for x in llg.DP45["bhat"]]
    for got, want in _order_conditions(A, bh, 4):
        assert got == want
    conds5 = _order_conditions(A, bh, 5)
    assert any(g != w for g, w in conds5)            # the embedded pair is not 5th order
    # FSAL: the last stage row equals b
    assert [Fraction(x).limit_denominator(10 ** 7) for x in llg.DP45["A"][6]] == \
        [Fraction(x).limit_denominator(10 ** 7) for x in llg.DP45["b"][:6]]


def test_norm_drift_without_renormalisation_is_high_order():
    """PIN-10b: with renormalisation off, |m| drifts by O(dt^(p+1)) per
    step (the exact flow conserves |m|)."""
    drifts = []
    for dt in (2e-13, 1e-13):
        prob, m0 = _macrospin(0.2, 0.5)
        s = llg.Solver(prob, m0, renormalize=False)
        s.step("rk4", dt, 1)
        drifts.append(abs(np.linalg.norm(s.m[:, 0, 0, 0]) - 1))
    assert math.log2(drifts[0] / drifts[1]) > 4.5


def test_energy_decays_with_damping_and_is_conserved_without():
    """PIN-13: with alpha > 0 and a static field the energy never rises; with
    alpha = 0 it is conserved to integrator error."""
    prob, m0 = workloads.small_problem(n=(12, 10, 1), alpha=0.5)
    s = llg.Solver(prob, m0)
    E = [fields.energy(s.m, prob)]
    for _ in range(40):
        s.step("rk4", 2e-14, 5)
        E.append(fields.energy(s.m, prob))
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E, E[1:]))
    assert E[-1] < E[0]
    prob0 = dict(prob, alpha=0.0)
    s = llg.Solver(prob0, m0)
    E0 = fields.energy(s.m, prob0)
    s.step("rk4", 5e-15, 100)
    assert abs(fields.energy(s.m, prob0) - E0) < 1e-6 * abs(E0)


def test_dp45_controller_and_replay():
    """Free-running DP45 reaches t_end exactly; replaying its own attempt log
    reproduces the trajectory bit for bit."""
    prob, m0 = workloads.small_problem(n=(6, 5, 1), alpha=0.3)
    a = llg.Solver(prob, m0)
    log = a.run_adaptive(2e-11, 1e-5, 1e-14)
    assert a.t == pytest.approx(2e-11, rel=1e-12)
    assert any(not ok for _, _, ok in log) or len(log) > 3
    b = llg.Solver(prob, m0)
    b.replay([(h, ok) for h, _, ok in log])
    assert np.array_equal(a.m, b.m)
    assert llg.Solver.next_dt(1.0, 0.0, 1e-5) == 5.0
    assert llg.Solver.next_dt(1.0, 1.0, 1e-5) == 0.2
    assert llg.Solver.next_dt(1.0, 1e-5, 1e-5) == pytest.approx(0.9)


@pytest.mark.parametrize("name,q,p", [("rk12", 1, 2), ("rk23", 2, 3), ("rkck", 4, 5)])
def test_embedded_estimates_have_their_order(name, q, p):
    """The embedded weights of each pair satisfy the order conditions up to
    q and fail one of order q + 1 (so the error estimate is of order q + 1
    in the step, as the controller assumes)."""
    tab = llg.ADAPTIVE[name][0]
    assert llg.ADAPTIVE[name][1] == q
    A, _ = _as_fractions(tab)
    bh = [Fraction(x).limit_denominator(10 ** 7) for x in tab["bhat"]]
    for got, want in _order_conditions(A, bh, q):
        assert got == want
    assert any(g != w for g, w in _order_conditions(A, bh, q + 1))


def test_rk23_is_first_same_as_last():
    tab = llg.RK23
    conv = lambda x: Fraction(x).limit_denominator(10 ** 7)
    assert [conv(x) for x in tab["A"][3]] == [conv(x) for x in tab["b"][:3]] and tab["b"][3] == 0.0


def test_adaptive_error_estimate_scales_with_its_order():
    """On the macrospin the per-step error estimate of each pair falls as
    dt^(q+1) when the step halves."""
    alpha, Bz = 0.2, 0.2
    for name, (tab, q) in llg.ADAPTIVE.items():
        errs = []
        for dt in (2e-13, 1e-13):
            prob, m0 = _macrospin(alpha, Bz)
            s = llg.Solver(prob, m0)
            errs.append(s.attempt(dt, name)[1])
        rate = math.log2(errs[0] / errs[1])
        assert abs(rate - (q + 1)) < 0.3, (name, errs, rate)


def test_controller_exponent_follows_the_pair():
    # err = tol * 2^(q+1): the next step halves (times the 0.9 safety factor)
    for q in (1, 2, 4):
        assert llg.Solver.next_dt(1.0, 2.0 ** (q + 1), 1.0, q) == pytest.approx(0.45)


@pytest.mark.parametrize("method,dt0,tol,t_end", [("rkdp45", 4e-12, 1e-5, 1e-10),
                                                  ("rkdp45", 2e-11, 1e-5, 1e-10),
                                                  ("rk23", 4e-13, 1e-6, 5e-11)])
def test_step_sequence_matches_scipy(method, dt0, tol, t_end):
    """PIN-12c: the adaptive driver (Sec. 2.2: embedded error per step,
    accept/reject, the step-size rule, the last step landing on t_end)
    against scipy's independent Dormand-Prince 5(4) and Bogacki-Shampine
    3(2) solvers on one tilted, anisotropic cell integrated without
    renormalisation.  With one cell the per-cell Euclidean error over tol
    equals scipy's RMS error norm with atol = tol/sqrt(3) (rtol at scipy's
    floor); both controllers then use 0.9 (tol/err)^(1/(q+1)).  They differ
    only where a factor leaves [0.2, 5] or a retry after a rejection would
    grow the step (scipy caps it at 1), so the cases are chosen, and checked
    here, to stay clear of both."""
    from scipy.integrate import RK23, RK45
    prob = dict(n=(1, 1, 1), cell=(5e-9,) * 3, pbc=(False,) * 3, Ms=8e5, Aex=1.3e-11,
                alpha=0.05, Ku=2e5, u=(0.6, 0.0, 0.8), B=(0.02, 0.0, 0.05), T=0.0, seed=0)
    th, ph = 1.2, 0.4
    m0 = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph),
                   math.cos(th)]).reshape(3, 1, 1, 1)
    s = llg.Solver(prob, m0, renormalize=False)
    q = llg.ADAPTIVE[method][1]
    log = s.run_adaptive(t_end, tol, dt0, method=method)
    fac = [0.9 * (tol / e) ** (1.0 / (q + 1)) for _, e, _ in log]
    assert all(0.2 < f < 5.0 for f in fac[:-1])
    assert all(fac[i + 1] <= 1.0 for i, (_, _, ok) in enumerate(log[:-1]) if not ok)
    t_ours = np.cumsum([h for h, _, ok in log if ok])

    f = lambda t, y: s.rhs(y.reshape(3, 1, 1, 1), None).reshape(3)
    ref = {"rkdp45": RK45, "rk23": RK23}[method](f, 0.0, m0.reshape(3).copy(), t_end,
                                                 first_step=dt0, rtol=1e-13,
                                                 atol=tol / math.sqrt(3.0))
    t_ref = []
    while ref.status == "running":
        ref.step()
        t_ref.append(ref.t)
    assert ref.status == "finished" and len(t_ref) == len(t_ours) > 10
    np.testing.assert_allclose(t_ours, t_ref, rtol=1e-7, atol=0.0)
    np.testing.assert_allclose(s.m.reshape(3), ref.y, rtol=0.0, atol=1e-10)


def _cubic_macrospin(K1, tilt, axis_kind):
    """One cubic cell with cubic anisotropy along rotated axes and strong
    damping, started `tilt` rad away from an easy axis."""
    rng = np.random.default_rng(11)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    c1, c2 = q[:, 0], q[:, 1]
    c3 = np.cross(c1, c2)
    easy = c1 if axis_kind == "100" else (c1 + c2 + c3) / math.sqrt(3.0)
    perp = np.cross(easy, rng.standard_normal(3))
    perp /= np.linalg.norm(perp)
    m0 = (math.cos(tilt) * easy + math.sin(tilt) * perp).reshape(3, 1, 1, 1)
    prob = dict(n=(1, 1, 1), cell=(5e-9,) * 3, pbc=(False,) * 3, Ms=8e5, Aex=1.3e-11, alpha=1.0,
                Ku=0.0, Kc1=K1, Kc2=0.0, c1=tuple(c1), c2=tuple(c2), B=(0.0, 0.0, 0.0), T=0.0, seed=0)
    return prob, m0, easy


@pytest.mark.parametrize("K1,kind", [(5e5, "100"), (-5e5, "111")])
def test_cubic_macrospin_relaxes_to_the_easy_axis(K1, kind):
    """Eq. 5: with K1 > 0 the easy axes are the cube axes c_i, with K1 < 0
    the body diagonals; a strongly damped single cell (isotropic self-demag,
    no other torque) relaxes onto the nearest one."""
    prob, m0, easy = _cubic_macrospin(K1, 0.4, kind)
    s = llg.Solver(prob, m0)
    s.step("rk4", 1e-13, 3000)
    np.testing.assert_allclose(s.m[:, 0, 0, 0], easy, atol=1e-6)


# --------------------------------------------------------------------------
# Zhang-Li spin-transfer torque (Eq. 7-8)
# --------------------------------------------------------------------------
MU_B, E_CHARGE = 9.2740100783e-24, 1.602176634e-19   # CODATA values


def _spiral(n, k_cells, xi, alpha, j=1e12, P=0.6):
    """In-plane spiral m = (cos q x, sin q x, 0), q = 2 pi k / (n dx), on a
    ring periodic in x, with no field term at all: only the current acts."""
    dx = 3e-9
    x = np.arange(n) * dx
    q = 2 * math.pi * k_cells / (n * dx)
    m0 = np.stack([np.cos(q * x), np.sin(q * x), np.zeros(n)]).reshape(3, 1, 1, n)
    prob = dict(n=(n, 1, 1), cell=(dx, dx, dx), pbc=(True, False, False), Ms=8e5, Aex=1.3e-11,
                alpha=alpha, terms=(), j=(j, 0.0, 0.0), P=P, xi=xi, T=0.0, seed=0)
    return prob, m0, q, dx


def test_stt_uniform_state_is_left_alone():
    prob, _, _, _ = _spiral(16, 1, 0.05, 0.1)
    m = workloads.uniform((16, 1, 1), (0.3, -0.5, 0.8)).astype(np.float64)
    assert np.max(np.abs(llg.stt_rhs(m, prob))) == 0.0


def test_stt_initial_rate_on_a_spiral():
    """dm/dt = b_j s / (1 + alpha^2) [e_theta - (xi - alpha) z] with
    s = j sin(q dx) / dx, the discrete central difference of the spiral."""
    alpha, xi, P, j = 0.1, 0.05, 0.6, 1e12
    prob, m0, q, dx = _spiral(24, 2, xi, alpha, j, P)
    bj = P * MU_B / (E_CHARGE * prob["Ms"] * (1 + xi * xi))
    s = j * math.sin(q * dx) / dx
    th = q * np.arange(24) * dx
    want = bj * s / (1 + alpha ** 2) * np.stack([-np.sin(th), np.cos(th), -(xi - alpha) * np.ones(24)])
    np.testing.assert_allclose(llg.stt_rhs(m0, prob).reshape(3, -1), want, rtol=1e-12,
                               atol=1e-12 * np.max(np.abs(want)))


def test_stt_adiabatic_spiral_rotates_rigidly():
    """With xi = alpha the spiral stays a spiral and every cell turns at the
    rate b_j s / (1 + alpha^2) (the discrete form of the rigid drift)."""
    alpha = xi = 0.1
    P, j, n = 0.6, 1e12, 24
    prob, m0, q, dx = _spiral(n, 2, xi, alpha, j, P)
    bj = P * MU_B / (E_CHARGE * prob["Ms"] * (1 + xi * xi))
    w = bj * j * math.sin(q * dx) / dx / (1 + alpha ** 2)
    o = llg.Solver(prob, m0)
    t = 2e-11
    o.step("rk4", 1e-13, 200)
    th = q * np.arange(n) * dx + w * t
    want = np.stack([np.cos(th), np.sin(th), np.zeros(n)])
    np.testing.assert_allclose(o.m.reshape(3, -1), want, atol=1e-9)


def test_dm_controller_macrospin_closed_form():
    """Bounded variation of m per step (Sec. 2.2) on an undamped macrospin:
    |dm/dt| = gamma0 H sin(theta0) all along the precession, so every step is
    max_dm / (gamma0 H sin theta0), the last one shortened to land on t_end,
    and RK4 along those steps follows the closed-form precession."""
    Bz, th0 = 0.1, 1.0
    prob, m0 = _macrospin(0.0, Bz, theta0=th0)
    s = llg.Solver(prob, m0)
    max_dm, t_end = 1e-2, 2e-10
    rec = s.run_dm("rk4", t_end, max_dm, dt_max=1e-9)
    h = max_dm / (GAMMA0 * Bz / MU0 * math.sin(th0))
    assert s.t == t_end
    assert len(rec) == math.ceil(t_end / h)
    for dt, own in rec[:-1]:
        assert dt == own
        assert dt == pytest.approx(h, rel=1e-9)
    assert rec[-1][0] == pytest.approx(t_end - (len(rec) - 1) * h, rel=1e-6)
    np.testing.assert_allclose(s.m[:, 0, 0, 0], _macrospin_exact(0.0, Bz, t_end, theta0=th0), atol=1e-8)


def test_dm_controller_first_step_with_damping_and_cap():
    """Damped macrospin: m x H and m x (m x H) are orthogonal and of equal
    length, so |dm/dt| = gamma0 H sin(theta0) / sqrt(1 + alpha^2) and the
    first step is max_dm sqrt(1 + alpha^2) / (gamma0 H sin theta0); dt_max
    caps it."""
    alpha, Bz, th0 = 0.5, 0.1, 1.0
    prob, m0 = _macrospin(alpha, Bz, theta0=th0)
    s = llg.Solver(prob, m0)
    dt, _ = s.dm_step(1e-2, 1.0, 1.0)
    assert dt == pytest.approx(1e-2 * math.sqrt(1 + alpha ** 2) / (GAMMA0 * Bz / MU0 * math.sin(th0)), rel=1e-12)
    assert s.dm_step(1e-2, 1e-13, 1.0)[0] == 1e-13
    assert s.dm_step(1e-2, 1.0, 1e-14)[0] == 1e-14          # time left
    still = llg.Solver(_macrospin(alpha, Bz, theta0=0.0)[0], np.array([0.0, 0.0, 1.0]).reshape(3, 1, 1, 1))
    assert still.dm_step(1e-2, 3e-12, 1.0)[0] == 3e-12      # no torque: the cap


def test_dm_controller_bounds_the_change_of_every_cell():
    """Euler on a random film: the torque is orthogonal to m, so a step of
    size dt |k| = d moves a cell by 2 - 2/sqrt(1 + d^2) squared, i.e. by at
    most d and by d (1 - O(d^2)) for the fastest cell, whose d is max_dm."""
    prob, m0 = workloads.small_problem(n=(8, 6, 1), alpha=0.5)
    s = llg.Solver(prob, m0)
    max_dm = 1e-2
    for _ in range(10):
        before = s.m.copy()
        dt, _ = s.dm_step(max_dm, 1e-9, 1.0)
        s.run_dm("euler", 1.0, max_dm, 1e-9, dts=[dt])
        d = np.sqrt(np.sum((s.m - before) ** 2, axis=0))
        assert d.max() <= max_dm * (1 + 1e-12)
        assert d.max() >= max_dm * (1 - max_dm ** 2)
