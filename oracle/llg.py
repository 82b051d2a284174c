"""Landau-Lifshitz right-hand side and Runge-Kutta time stepping, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2, Eq. 1 with M = Ms m:

    dm/dt = -gamma/(1+alpha^2) m x H  -  alpha gamma/(1+alpha^2) m x (m x H)

Sec. 2.2 lists the explicit Runge-Kutta schemes.  Every stage input and every
accepted state is renormalised to |m| = 1 (the paper is silent on this; the
exact flow keeps |m| = 1, and normalising the stage inputs is the same as
integrating dm/dt = f(m/|m|), so the order of each scheme is kept).  The
thermal field of Eq. 6 is drawn once per step and held fixed across the
stages of that step.

Adaptive embedded pairs of Sec. 2.2 (Dormand-Prince 5(4), Bogacki-Shampine
3(2), Cash-Karp 5(4), Heun-Euler 2(1)), with the reading of the "maximum
tolerable error per integration step":
    err  = max over cells |dt sum_j (b_j - bhat_j) k_j|
    accept if err <= tol
    dt  <- dt * clamp(0.9 (tol/err)^(1/(q+1)), 0.2, 5)  (5 if err == 0),
           q the order of the embedded estimate
    the last step is shortened to land on t_end.

The fixed schemes may instead bound the variation of m per step (Sec. 2.2),
read here as: before each step, dt = max_dm / max over cells |dm/dt| at the
current state (the step's first stage), at most dt_max, the last step
shortened to land on t_end; the thermal term is left out (its strength
depends on a fixed step).
"""
import math

import numpy as np

from .constants import GAMMA0, MU_B, E_CHARGE
from . import fields

# --------------------------------------------------------------------------
# Butcher tableaux (c implied by row sums)
# --------------------------------------------------------------------------
EULER = {"A": [[]], "b": [1.0]}
HEUN = {"A": [[], [1.0]], "b": [0.5, 0.5]}
RK4 = {"A": [[], [0.5], [0.0, 0.5], [0.0, 0.0, 1.0]],
       "b": [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]}
# Dormand & Prince (1980), RK5(4)7M
DP45 = {
    "A": [
        [],
        [1.0 / 5.0],
        [3.0 / 40.0, 9.0 / 40.0],
        [44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0],
        [19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0],
        [9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0],
        [35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0],
    ],
    "b": [35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0],
    "bhat": [5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0, -92097.0 / 339200.0,
             187.0 / 2100.0, 1.0 / 40.0],
}
# Kutta's third-order method
RK3 = {"A": [[], [0.5], [-1.0, 2.0]], "b": [1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0]}
# Heun-Euler 2(1): Heun's method with Euler's as the embedded estimate
RK12 = {"A": [[], [1.0]], "b": [0.5, 0.5], "bhat": [1.0, 0.0]}
# Bogacki & Shampine (1989), 3(2) with the first-same-as-last property
RK23 = {
    "A": [[], [0.5], [0.0, 0.75], [2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0]],
    "b": [2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0, 0.0],
    "bhat": [7.0 / 24.0, 0.25, 1.0 / 3.0, 0.125],
}
# Cash & Karp (1990), 5(4)
RKCK = {
    "A": [
        [],
        [0.2],
        [3.0 / 40.0, 9.0 / 40.0],
        [0.3, -0.9, 1.2],
        [-11.0 / 54.0, 2.5, -70.0 / 27.0, 35.0 / 27.0],
        [1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0],
    ],
    "b": [37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0],
    "bhat": [2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0, 277.0 / 14336.0, 0.25],
}
TABLEAUX = {"euler": EULER, "heun": HEUN, "rk3": RK3, "rk4": RK4, "rkdp45": DP45,
            "rk12": RK12, "rk23": RK23, "rkck": RKCK}
# adaptive pairs: (tableau, order of the embedded estimate q); the step
# controller uses the exponent 1/(q+1)
ADAPTIVE = {"rkdp45": (DP45, 4), "rk23": (RK23, 2), "rkck": (RKCK, 4), "rk12": (RK12, 1)}


def normalize(m):
    return m / np.sqrt(np.sum(m * m, axis=0, keepdims=True))


def ll_rhs(m, H, alpha):
    """Eq. 1 divided by Ms: dm/dt for field H (A/m)."""
    mxH = np.cross(m, H, axis=0)
    mxmxH = np.cross(m, mxH, axis=0)
    return -GAMMA0 / (1.0 + alpha * alpha) * (mxH + alpha * mxmxH)


def current_gradient(m, prob):
    """(j . grad) m with central differences per axis, (m[i+1] - m[i-1]) /
    (2 d); at a free surface the missing neighbour is the cell itself, a
    periodic axis wraps, an axis one cell long contributes nothing."""
    j = np.asarray(prob.get("j", (0.0, 0.0, 0.0)), dtype=np.float64)
    D = np.zeros_like(m)
    for a, axis in ((0, 3), (1, 2), (2, 1)):
        n = m.shape[axis]
        if j[a] == 0.0 or n == 1:
            continue
        up = np.roll(m, -1, axis=axis)     # neighbour at index i+1
        dn = np.roll(m, 1, axis=axis)      # neighbour at index i-1
        if not prob["pbc"][a]:
            last = [slice(None)] * 4
            last[axis] = n - 1
            up[tuple(last)] = m[tuple(last)]
            first = [slice(None)] * 4
            first[axis] = 0
            dn[tuple(first)] = m[tuple(first)]
        D += j[a] * (up - dn) / (2.0 * prob["cell"][a])
    return D


def stt_rhs(m, prob):
    """Sec. 2.1.3, Eq. 7-8 divided by Ms: the Zhang-Li terms
    -b_j/(1+alpha^2) [m x (m x D) + (xi - alpha) m x D], D = (j . grad) m,
    b_j = P mu_B / (e Ms (1 + xi^2))."""
    j = np.asarray(prob.get("j", (0.0, 0.0, 0.0)), dtype=np.float64)
    if not np.any(j):
        return np.zeros_like(m)
    alpha, xi, P = prob["alpha"], prob.get("xi", 0.0), prob.get("P", 0.0)
    bj = P * MU_B / (E_CHARGE * prob["Ms"] * (1.0 + xi * xi))
    D = current_gradient(m, prob)
    mxD = np.cross(m, D, axis=0)
    mxmxD = np.cross(m, mxD, axis=0)
    return -bj / (1.0 + alpha * alpha) * (mxmxD + (xi - alpha) * mxD)


class Solver:
    """Plain FP64 integrator state for one problem."""

    def __init__(self, prob, m0, renormalize=True):
        self.prob = dict(prob)
        # the library renormalises the state it is given; so does the oracle
        self.m = normalize(np.array(m0, dtype=np.float64)) if renormalize \
            else np.array(m0, dtype=np.float64)
        self.t = 0.0
        self.step_count = 0          # accepted steps: thermal draw counter
        self.evals = 0
        self.renormalize = renormalize

    # -- field and derivative -------------------------------------------------
    def rhs(self, m, dt):
        H = fields.heff(m, self.prob, dt=dt, step=self.step_count)
        self.evals += 1
        return ll_rhs(m, H, self.prob["alpha"]) + stt_rhs(m, self.prob)

    def _norm(self, m):
        return normalize(m) if self.renormalize else m

    def _stages(self, tab, dt, k1=None):
        """Runs the stages of one explicit RK step from self.m; returns k.
        A given k1 (f at self.m) is used instead of evaluating it again."""
        ks = []
        for s, row in enumerate(tab["A"]):
            if s == 0 and k1 is not None:
                ks.append(k1)
                continue
            if s == 0:
                ms = self.m
            else:
                ms = self.m.copy()
                for a, k in zip(row, ks):
                    if a != 0.0:
                        ms = ms + (dt * a) * k
                ms = self._norm(ms)
            ks.append(self.rhs(ms, dt))
        return ks

    def _combine(self, ks, weights, dt):
        out = self.m.copy()
        for w, k in zip(weights, ks):
            if w != 0.0:
                out = out + (dt * w) * k
        return out

    # -- fixed step -----------------------------------------------------------
    def step(self, method, dt, nsteps=1):
        tab = TABLEAUX[method]
        for _ in range(nsteps):
            ks = self._stages(tab, dt)
            self.m = self._norm(self._combine(ks, tab["b"], dt))
            self.t += dt
            self.step_count += 1
        return self.m

    # -- fixed tableau, step bounded by the variation of m -----------------------
    def dm_step(self, max_dm, dt_max, t_end):
        """(dt, k1) for the next step: k1 = f(m), dt = max_dm / max_i |k1_i|
        limited to dt_max and to the time left."""
        k1 = self.rhs(self.m, None)
        kmax = float(np.max(np.sqrt(np.sum(k1 * k1, axis=0))))
        dt = dt_max if kmax == 0.0 else min(dt_max, max_dm / kmax)
        return min(dt, t_end - self.t), k1

    def run_dm(self, method, t_end, max_dm, dt_max, dts=None):
        """Integrates to t_end with the fixed tableau `method`, each step
        chosen by dm_step.  With `dts` (a recorded list of steps, e.g. the
        GPU run's) those steps are taken instead.  Returns [(dt taken, dt the
        oracle chose)] per step."""
        tab = TABLEAUX[method]
        saved = self.prob
        self.prob = dict(saved, T=0.0)
        out = []
        try:
            while (self.t < t_end) if dts is None else (len(out) < len(dts)):
                own, k1 = self.dm_step(max_dm, dt_max, t_end)
                dt = own if dts is None else dts[len(out)]
                ks = self._stages(tab, dt, k1)
                self.m = self._norm(self._combine(ks, tab["b"], dt))
                self.t = t_end if dt >= t_end - self.t else self.t + dt
                self.step_count += 1
                out.append((dt, own))
        finally:
            self.prob = saved
        return out

    # -- adaptive embedded pairs (Dormand-Prince by default) --------------------
    def attempt(self, dt, method="rkdp45"):
        """One attempted step of an embedded pair: returns (candidate m, err)
        with err = max over cells |dt sum_j (b_j - bhat_j) k_j|."""
        tab = ADAPTIVE[method][0]
        ks = self._stages(tab, dt)
        m_hi = self._combine(ks, tab["b"], dt)
        diff = np.zeros_like(self.m)
        for b, bh, k in zip(tab["b"], tab["bhat"], ks):
            if b != bh:
                diff = diff + (dt * (b - bh)) * k
        err = float(np.max(np.sqrt(np.sum(diff * diff, axis=0))))
        return self._norm(m_hi), err

    def dp45_attempt(self, dt):
        return self.attempt(dt, "rkdp45")

    @staticmethod
    def next_dt(dt, err, tol, q=4):
        """dt * clamp(0.9 (tol/err)^(1/(q+1)), 0.2, 5) for an embedded
        estimate of order q."""
        if err == 0.0:
            factor = 5.0
        else:
            factor = 0.9 * (tol / err) ** (1.0 / (q + 1))
        return dt * min(5.0, max(0.2, factor))

    def run_adaptive(self, t_end, tol, dt0, dt_min=1e-18, max_attempts=10 ** 7, method="rkdp45"):
        """Free-running adaptive integration to t_end; returns the list of
        attempts (dt, err, accepted)."""
        q = ADAPTIVE[method][1]
        log = []
        dt = dt0
        while self.t < t_end and len(log) < max_attempts:
            h = min(dt, t_end - self.t)
            m_new, err = self.attempt(h, method)
            ok = err <= tol
            log.append((h, err, ok))
            if ok:
                self.m = m_new
                self.t += h
                self.step_count += 1
            dt = self.next_dt(h, err, tol, q)
            if dt < dt_min:
                raise FloatingPointError("step size fell below dt_min")
        return log

    def replay(self, attempts, method="rkdp45"):
        """Replays a recorded attempt list [(dt, accepted), ...] (e.g. the GPU
        run's), so both trajectories use the same step sizes; returns the
        oracle's own error estimate per attempt."""
        errs = []
        for dt, ok in attempts:
            m_new, err = self.attempt(dt, method)
            errs.append(err)
            if ok:
                self.m = m_new
                self.t += dt
                self.step_count += 1
        return errs
