"""Seeded synthetic inputs for the solver and the oracle.

This module only generates inputs (problem parameters and initial
magnetisation arrays).  It holds none of the method's arithmetic, so both the
GPU library's callers and the FP64 oracle may use it.

Problems are dicts in SI units (see ``oracle.fields`` for the keys); initial
states are float32 arrays of shape (3, nz, ny, nx), x fastest, unit vectors
per cell.  The float32 values are what the GPU receives; the oracle promotes
the very same values to float64.

The workloads follow the shapes of the paper's runs: thin films of
permalloy-like material (Ms = 8e5 A/m, A = 1.3e-11 J/m) with the thickness,
damping and applied field of muMAG standard problem 4 (Sec. 4.2 of the paper,
"field 1"), enlarged to a 512 x 512 cell film; no data from that benchmark
(reference solutions) is used or needed.
"""
import math

import numpy as np


def random_unit(n, seed):
    """Uniform random directions: three standard normals per cell, scaled to
    unit length."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((3, nz, ny, nx))
    g /= np.sqrt(np.sum(g * g, axis=0, keepdims=True))
    return g.astype(np.float32)


def uniform(n, direction):
    nx, ny, nz = n
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    return np.broadcast_to(d.reshape(3, 1, 1, 1), (3, nz, ny, nx)).astype(np.float32).copy()


def vortex(n, core_radius):
    """In-plane curl with a +z core of the given radius (cells), centred on
    the film's geometric centre; identical in every z layer."""
    nx, ny, nz = n
    x = np.arange(nx) + 0.5 - nx / 2.0
    y = np.arange(ny) + 0.5 - ny / 2.0
    X, Y = np.meshgrid(x, y, indexing="xy")
    r = np.hypot(X, Y)
    phi = np.arctan2(Y, X)
    theta = np.where(r < core_radius, 0.5 * math.pi * r / core_radius, 0.5 * math.pi)
    m = np.stack([-np.sin(phi) * np.sin(theta), np.cos(phi) * np.sin(theta), np.cos(theta)])
    m = np.broadcast_to(m[:, None], (3, nz, ny, nx))
    return m.astype(np.float32).copy()


def field_in_plane(b_tesla, angle_deg):
    a = math.radians(angle_deg)
    return (b_tesla * math.cos(a), b_tesla * math.sin(a), 0.0)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def film_32():
    """32x32x1 cells of 4 nm cubes, random start, strong damping; fixed-step
    Heun and RK4 at dt = 1e-13 s for 1000 steps."""
    n = (32, 32, 1)
    prob = dict(n=n, cell=(4e-9, 4e-9, 4e-9), pbc=(False, False, False),
                Ms=8.0e5, Aex=1.3e-11, alpha=0.5, Ku=0.0, u=(1.0, 0.0, 0.0),
                B=(0.0, 0.0, 0.0), T=0.0, seed=0)
    run = dict(methods=("heun", "rk4"), dt=1e-13, steps=1000)
    return prob, random_unit(n, 1), run


def film_512(n_side=512):
    """Thin film n x n x 1 of 4x4x3 nm cells, alpha 0.02, uniaxial
    anisotropy 5e3 J/m^3 along x, 25 mT applied at 170 degrees in plane,
    start along (1,1,1)/sqrt(3); adaptive Dormand-Prince to 1 ns."""
    n = (n_side, n_side, 1)
    prob = dict(n=n, cell=(4e-9, 4e-9, 3e-9), pbc=(False, False, False),
                Ms=8.0e5, Aex=1.3e-11, alpha=0.02, Ku=5.0e3, u=(1.0, 0.0, 0.0),
                B=field_in_plane(0.025, 170.0), T=0.0, seed=0)
    run = dict(methods=("rkdp45",), t_end=1e-9, tol=1e-5, dt0=1e-14)
    return prob, uniform(n, (1.0, 1.0, 1.0)), run


def film_3d(n=(256, 256, 64)):
    """3D block of 3 nm cubes, periodic in x and y, 300 K thermal field,
    vortex start with a 10-cell core; Heun at dt = 5e-14 s."""
    prob = dict(n=n, cell=(3e-9, 3e-9, 3e-9), pbc=(True, True, False), images=10,
                Ms=1.0e6, Aex=1.5e-11, alpha=0.1, Ku=0.0, u=(1.0, 0.0, 0.0),
                B=(0.0, 0.0, 0.0), T=300.0, seed=3)
    run = dict(methods=("heun",), dt=5e-14, steps=10000)
    return prob, vortex(n, 10.0), run


def film_batch(nfilms=64, seed=4, sizes=(64, 96, 128, 192, 256)):
    """Independent square films of uneven size from a parameter sweep."""
    rng = np.random.default_rng(seed)
    films = []
    for f in range(nfilms):
        side = int(rng.choice(sizes))
        n = (side, side, 1)
        Ms = float(rng.uniform(6e5, 1.2e6))
        alpha = float(rng.uniform(0.01, 0.5))
        b = float(rng.uniform(0.0, 0.1))
        ang = float(rng.uniform(0.0, 360.0))
        prob = dict(n=n, cell=(4e-9, 4e-9, 3e-9), pbc=(False, False, False),
                    Ms=Ms, Aex=1.3e-11, alpha=alpha, Ku=0.0, u=(1.0, 0.0, 0.0),
                    B=field_in_plane(b, ang), T=0.0, seed=0)
        m0 = random_unit(n, int(rng.integers(1 << 31)))
        films.append((prob, m0))
    run = dict(methods=("rkdp45",), t_end=0.5e-9, tol=1e-5, dt0=1e-14)
    return films, run


def sp2_films(count=200, r_min=1.0, r_max=30.0, max_width=64):
    """Films shaped like the static standard problem of Sec. 4.1: a cuboid of
    5d x d x 0.1d with only demag and exchange, saturated along [1,1,1] at
    the start and relaxed with alpha = 1, for `count` values of d/l_ex evenly
    spaced in [r_min, r_max] (l_ex = sqrt(2A/(mu0 Ms^2)), 5.7 nm for the
    material used here; only d/l_ex matters).  Cells: ny = clamp(ceil(2 d/l_ex),
    4, max_width) across the width, so the cell edge stays at or below half
    the exchange length up to d/l_ex = max_width/2; nx = 5 ny; one cell
    through the thickness.  The paper ran 200 such relaxations."""
    Ms, A = 8.0e5, 1.3e-11
    lex = math.sqrt(2.0 * A / (4e-7 * math.pi * Ms * Ms))
    films = []
    for k in range(count):
        r = r_min + (r_max - r_min) * k / max(count - 1, 1)
        d = r * lex
        ny = min(max(int(math.ceil(2.0 * r)), 4), max_width)
        nx = 5 * ny
        c = d / ny
        prob = dict(n=(nx, ny, 1), cell=(c, c, 0.1 * d), pbc=(False, False, False), Ms=Ms, Aex=A,
                    alpha=1.0, Ku=0.0, u=(1.0, 0.0, 0.0), B=(0.0, 0.0, 0.0), T=0.0, seed=0, d_over_lex=r)
        films.append((prob, uniform((nx, ny, 1), (1.0, 1.0, 1.0))))
    run = dict(methods=("rkdp45",), t_end=1e-9, tol=1e-5, dt0=1e-14)
    return films, run


def surrogate_films(ntraj, seed=5, n_side=256):
    """Trajectories for the learned surrogate: the thin film of film_512 at
    n x n cells, each with its own applied field of magnitude U[0, 50] mT at
    a uniformly random in-plane angle, all starting along (1,1,1)/sqrt(3).
    Pairs (m_t, m_t+10 steps) come from fixed RK4 steps of 1e-13 s after a
    50-step burn-in, one pair every 10 steps."""
    rng = np.random.default_rng(seed)
    prob0, m0, _ = film_512(n_side)
    films = []
    for _ in range(ntraj):
        prob = dict(prob0)
        prob["B"] = field_in_plane(float(rng.uniform(0.0, 0.05)), float(rng.uniform(0.0, 360.0)))
        films.append((prob, m0.copy()))
    run = dict(method="rk4", dt=1e-13, seg_steps=10, burn_in=50)
    return films, run


SURROGATE_LAYERS = ((9, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3))


def surrogate_init(seed=0):
    """Seeded initial weights of the surrogate network, list of (w, b) per
    layer with w of shape (cout, cin, 3, 3): normal with std sqrt(2 / (9
    cin)) (the last layer ten times smaller, so the first proposals are
    close to "no change"), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for li, (ci, co) in enumerate(SURROGATE_LAYERS):
        std = np.sqrt(2.0 / (9 * ci))
        if li == len(SURROGATE_LAYERS) - 1:
            std *= 0.1
        params.append((rng.standard_normal((co, ci, 3, 3)) * std, np.zeros(co)))
    return params


def small_problem(n=(8, 6, 1), cell=(4e-9, 4e-9, 3e-9), pbc=(False, False, False), seed=7,
                  **over):
    """A small random problem with every deterministic term switched on,
    for parity tests that must finish in seconds on the CPU."""
    rng = np.random.default_rng(seed)
    prob = dict(n=tuple(n), cell=tuple(cell), pbc=tuple(pbc), images=3,
                Ms=8.0e5, Aex=1.3e-11, alpha=0.1, Ku=5.0e3,
                u=tuple(_unit(rng.standard_normal(3))),
                B=tuple(rng.uniform(-0.05, 0.05, 3)), T=0.0, seed=0)
    prob.update(over)
    return prob, random_unit(n, seed + 1)


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)
