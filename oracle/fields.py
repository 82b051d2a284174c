"""Effective-field terms and energy, FP64, SI units.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A problem is a dict:

    n      = (nx, ny, nz)            cells
    cell   = (dx, dy, dz)            m
    pbc    = (px, py, pz)            bools
    images = P                       periodic images per periodic axis
    Ms, Aex, alpha                   A/m, J/m, 1
    Ku, u                            J/m^3, unit axis (uniaxial anisotropy)
    Kc1, Kc2, c1, c2                 J/m^3 and two orthogonal unit axes
                                     (cubic anisotropy; c3 = c1 x c2)
    B                                applied field mu0*H in tesla (3,)
    T, seed                          K, 64-bit seed (thermal field)
    terms                            subset of {"demag", "exchange",
                                     "anisotropy", "zeeman", "thermal"}

m has shape (3, nz, ny, nx) and is a unit vector per cell.
"""
import math

import numpy as np

from . import demag
from .constants import MU0, GAMMA0, KB
from .philox import thermal_eta

ALL_TERMS = ("demag", "exchange", "anisotropy", "zeeman", "thermal")


def geom_of(prob):
    return {"n": tuple(prob["n"]), "cell": tuple(prob["cell"]), "pbc": tuple(prob["pbc"]),
            "images": prob.get("images", demag.DEFAULT_IMAGES)}


def exchange_field(m, prob):
    """Sec. 2.1.2, Eq. 3: H_ex = (2A/(mu0 Ms)) lap m with the six-neighbour
    Laplacian sum_{axes, +/-} (m_nb - m)/d^2; a missing neighbour at a free
    surface is omitted (zero normal derivative), a periodic axis wraps.
    With one cell along z there are no z neighbours (the 4-neighbour case)."""
    m = np.asarray(m, dtype=np.float64)
    lap = np.zeros_like(m)
    dx, dy, dz = prob["cell"]
    for axis, d, per in ((3, dx, prob["pbc"][0]), (2, dy, prob["pbc"][1]), (1, dz, prob["pbc"][2])):
        n = m.shape[axis]
        for shift in (1, -1):
            nb = np.roll(m, shift, axis=axis)
            diff = (nb - m) / (d * d)
            if not per:
                # np.roll(+1) brings in the cell at index i-1; the cell at index
                # 0 has no such neighbour (and likewise index n-1 for -1).
                edge = [slice(None)] * 4
                edge[axis] = 0 if shift == 1 else n - 1
                diff[tuple(edge)] = 0.0
            lap += diff
    return 2.0 * prob["Aex"] / (MU0 * prob["Ms"]) * lap


def uniaxial_field(m, prob):
    """Sec. 2.1.3, Eq. 4: energy density Ku sin^2(theta) = Ku (1 - (m.u)^2);
    H = (2 Ku/(mu0 Ms)) (m.u) u."""
    u = np.asarray(prob.get("u", (1.0, 0.0, 0.0)), dtype=np.float64)
    u = u / np.linalg.norm(u)
    mu = np.tensordot(u, m, axes=(0, 0))
    return 2.0 * prob.get("Ku", 0.0) / (MU0 * prob["Ms"]) * mu[None] * u.reshape(3, 1, 1, 1)


def cubic_axes(prob):
    c1 = np.asarray(prob.get("c1", (1.0, 0.0, 0.0)), dtype=np.float64)
    c2 = np.asarray(prob.get("c2", (0.0, 1.0, 0.0)), dtype=np.float64)
    c1 = c1 / np.linalg.norm(c1)
    c2 = c2 / np.linalg.norm(c2)
    return c1, c2, np.cross(c1, c2)


def cubic_field(m, prob):
    """Sec. 2.1.3, Eq. 5: energy density K1 (a1^2 a2^2 + a2^2 a3^2 + a1^2 a3^2)
    + K2 a1^2 a2^2 a3^2 with a_i = m.c_i; H = -(1/(mu0 Ms)) dE/dm."""
    K1, K2 = prob.get("Kc1", 0.0), prob.get("Kc2", 0.0)
    cs = cubic_axes(prob)
    a = [np.tensordot(c, m, axes=(0, 0)) for c in cs]
    a2 = [x * x for x in a]
    H = np.zeros_like(m)
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        dEda = 2.0 * a[i] * (K1 * (a2[j] + a2[k]) + K2 * a2[j] * a2[k])
        H -= dEda[None] * cs[i].reshape(3, 1, 1, 1)
    return H / (MU0 * prob["Ms"])


def zeeman_field(m, prob):
    """Applied field H = B / mu0 (B given as mu0 H in tesla)."""
    B = np.asarray(prob.get("B", (0.0, 0.0, 0.0)), dtype=np.float64)
    return np.broadcast_to((B / MU0).reshape(3, 1, 1, 1), m.shape).copy()


def thermal_sigma(prob, dt):
    """Sec. 2.1.3, Eq. 6: sqrt(2 alpha k_B T / (gamma mu0 Ms V dt)), A/m."""
    dx, dy, dz = prob["cell"]
    V = dx * dy * dz
    return math.sqrt(2.0 * prob["alpha"] * KB * prob.get("T", 0.0) /
                     (GAMMA0 * MU0 * prob["Ms"] * V * dt))


def thermal_field(m, prob, dt, step):
    """eta * sigma with eta from the Philox draw of this step."""
    n = m[0].size
    eta = thermal_eta(n, step, int(prob.get("seed", 0)))
    return thermal_sigma(prob, dt) * eta.reshape(m.shape)


def terms_of(prob):
    t = prob.get("terms")
    return ALL_TERMS if t is None else tuple(t)


def heff_terms(m, prob, dt=None, step=0):
    """Dict of the enabled field terms (A/m)."""
    m = np.asarray(m, dtype=np.float64)
    out = {}
    terms = terms_of(prob)
    if "demag" in terms:
        out["demag"] = demag.demag_field_fft(m, prob["Ms"], geom_of(prob))
    if "exchange" in terms and prob.get("Aex", 0.0) != 0.0:
        out["exchange"] = exchange_field(m, prob)
    if "anisotropy" in terms:
        if prob.get("Ku", 0.0) != 0.0:
            out["anisotropy"] = uniaxial_field(m, prob)
        if prob.get("Kc1", 0.0) != 0.0 or prob.get("Kc2", 0.0) != 0.0:
            out["cubic"] = cubic_field(m, prob)
    if "zeeman" in terms:
        out["zeeman"] = zeeman_field(m, prob)
    if "thermal" in terms and prob.get("T", 0.0) > 0.0:
        if dt is None:
            raise ValueError("thermal field needs the time step")
        out["thermal"] = thermal_field(m, prob, dt, step)
    return out


def heff(m, prob, dt=None, step=0):
    """Total effective field, the sum of the enabled terms."""
    m = np.asarray(m, dtype=np.float64)
    H = np.zeros_like(m)
    for v in heff_terms(m, prob, dt, step).values():
        H = H + v
    return H


def energy_terms(m, prob):
    """Energies (J) whose negative gradient, divided by mu0 Ms V, is the
    field of the same term."""
    m = np.asarray(m, dtype=np.float64)
    dx, dy, dz = prob["cell"]
    V = dx * dy * dz
    Ms = prob["Ms"]
    out = {}
    terms = terms_of(prob)
    if "demag" in terms:
        Hd = demag.demag_field_fft(m, Ms, geom_of(prob))
        out["demag"] = -0.5 * MU0 * Ms * V * float(np.sum(m * Hd))
    if "exchange" in terms:
        e = 0.0
        for axis, d, per in ((3, dx, prob["pbc"][0]), (2, dy, prob["pbc"][1]), (1, dz, prob["pbc"][2])):
            n = m.shape[axis]
            if n == 1 and not per:
                continue
            nb = np.roll(m, -1, axis=axis)          # neighbour at index i+1
            sq = np.sum((nb - m) ** 2, axis=0)
            if not per:
                edge = [slice(None)] * 3
                edge[axis - 1] = n - 1
                sq[tuple(edge)] = 0.0
            e += float(np.sum(sq)) / (d * d)
        out["exchange"] = prob["Aex"] * V * e
    if "anisotropy" in terms:
        if prob.get("Ku", 0.0) != 0.0:
            u = np.asarray(prob.get("u", (1.0, 0.0, 0.0)), dtype=np.float64)
            u = u / np.linalg.norm(u)
            mu = np.tensordot(u, m, axes=(0, 0))
            out["anisotropy"] = prob["Ku"] * V * float(np.sum(1.0 - mu * mu))
        if prob.get("Kc1", 0.0) != 0.0 or prob.get("Kc2", 0.0) != 0.0:
            cs = cubic_axes(prob)
            a2 = [np.tensordot(c, m, axes=(0, 0)) ** 2 for c in cs]
            dens = prob.get("Kc1", 0.0) * (a2[0] * a2[1] + a2[1] * a2[2] + a2[0] * a2[2]) \
                + prob.get("Kc2", 0.0) * a2[0] * a2[1] * a2[2]
            out["cubic"] = V * float(np.sum(dens))
    if "zeeman" in terms:
        Hz = zeeman_field(m, prob)
        out["zeeman"] = -MU0 * Ms * V * float(np.sum(m * Hz))
    return out


def energy(m, prob):
    return sum(energy_terms(m, prob).values())
