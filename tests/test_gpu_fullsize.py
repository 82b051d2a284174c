"""Checks at the full sizes of the workloads, in the launch configuration the
benchmark uses, where the FP64 oracle cannot evaluate the whole problem in
seconds: properties that hold at any size (translation equivariance on
periodic axes, the exchange of a periodic spiral in closed form, uniform
states, reproducible thermal draws), sampled films replayed by the oracle,
and the surrogate's convolutions on a full 256 x 256 film."""
import math
import sys

import numpy as np
import pytest

import workloads
from oracle import fields, llg as ollg
from oracle import surrogate as osg
from oracle.constants import MU0

pytestmark = pytest.mark.gpu


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(3, -1)
    b = np.asarray(b, dtype=np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


def note(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def block(terms=None, T=0.0):
    """The 256 x 256 x 64 periodic block of the 3D workload."""
    prob, m0, run = workloads.film_3d()
    prob = dict(prob, T=T)
    if terms is not None:
        prob["terms"] = terms
    return prob, m0, run


def solver(lib, prob, m0):
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    return s


def test_block_translation_equivariance(lib):
    """x and y are periodic: shifting m by (5, -3) cells shifts H_eff (every
    deterministic term) by the same amount, to FP32 rounding."""
    prob, m0, _ = block()
    note("case: 256x256x64 periodic block, vortex, all deterministic terms")
    s = solver(lib, prob, m0)
    h0 = s.eval_heff()
    shifted = np.roll(m0, (-3, 5), axis=(2, 3)).copy()
    s.set_m(shifted)
    h1 = s.eval_heff()
    e = maxrel(h1, np.roll(h0, (-3, 5), axis=(2, 3)))
    note("translation: maxrel", e)
    assert e <= 1e-5


def test_block_spiral_exchange_closed_form(lib):
    """Exchange of m = (cos kx, sin kx, 0) with k = 2 pi 3 / (N dx) on the
    periodic x axis: H_ex = -(2A/(mu0 Ms)) (2 - 2 cos k dx)/dx^2 m exactly,
    at the full block size."""
    prob, _, _ = block(terms=("exchange",))
    nx, ny, nz = prob["n"]
    dx = prob["cell"][0]
    k = 2 * math.pi * 3 / (nx * dx)
    x = (np.arange(nx) + 0.5) * dx
    m = np.zeros((3, nz, ny, nx), np.float32)
    m[0] = np.cos(k * x)[None, None, :]
    m[1] = np.sin(k * x)[None, None, :]
    s = solver(lib, prob, m)
    h = s.eval_heff()
    want = -(2 * prob["Aex"] / (MU0 * prob["Ms"])) * (2 - 2 * math.cos(k * dx)) / dx ** 2 * m.astype(np.float64)
    e = float(np.max(np.abs(h - want))) / float(np.max(np.abs(want)))
    note("spiral exchange: max error / max field", e)
    assert e <= 1e-4


def test_block_uniform_state(lib):
    """Uniform m along (1, 2, 3)/|.|: the exchange field vanishes, and the
    demag field of the periodic slab does not depend on x or y (it varies
    only with z) and has no in-plane component for m along z."""
    prob, _, _ = block(terms=("demag", "exchange"))
    n = prob["n"]
    m = workloads.uniform(n, (1.0, 2.0, 3.0))
    s = solver(lib, prob, m)
    h = s.eval_heff().astype(np.float64)
    ref = h[:, :, :1, :1]
    spread = float(np.max(np.abs(h - ref))) / float(np.max(np.abs(h)))
    note("uniform state: in-plane spread of H / max H", spread)
    assert spread <= 1e-5
    s.set_m(workloads.uniform(n, (0.0, 0.0, 1.0)))
    hz = s.eval_heff().astype(np.float64)
    inplane = float(np.max(np.abs(hz[:2]))) / float(np.max(np.abs(hz[2])))
    note("m along z: in-plane H / max |H_z|", inplane, "H_z range", float(hz[2].min()), float(hz[2].max()))
    assert inplane <= 1e-5
    assert np.all(hz[2] < 0) and np.all(hz[2] > -prob["Ms"])


def test_block_thermal_heun_steps(lib):
    """Thermal Heun steps at full size: the same seed gives the same state
    bit for bit, another seed another state, and m stays of unit length."""
    prob, m0, run = block(T=300.0)
    a = solver(lib, prob, m0)
    a.step("heun", run["dt"], 3)
    b = solver(lib, prob, m0)
    b.step("heun", run["dt"], 3)
    ma = a.get_m()
    assert np.array_equal(ma, b.get_m())
    c = solver(lib, dict(prob, seed=4), m0)
    c.step("heun", run["dt"], 3)
    assert not np.array_equal(ma, c.get_m())
    norms = np.linalg.norm(ma.reshape(3, -1).astype(np.float64), axis=0)
    assert np.max(np.abs(norms - 1.0)) <= 1e-6


def test_sweep_films_replayed_by_oracle(lib):
    """The 64-film sweep at full size: its smallest and largest films,
    replayed by the oracle along their recorded attempts, match to 1e-5."""
    films, run = workloads.film_batch()
    b = lib.Batch(films)
    b.run(run["t_end"], run["tol"], run["dt0"], max_attempts=5)
    sides = [p["n"][0] for p, _ in films]
    for i in (int(np.argmin(sides)), int(np.argmax(sides))):
        prob, m0 = films[i]
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in b.attempts(i)])
        e = maxrel(b.get_m(i), o.m)
        note("sweep film", i, prob["n"], "m maxrel vs oracle", e)
        assert e <= 1e-5


def bf16(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def test_surrogate_layer_on_full_film(lib):
    """One 32 -> 32 convolution of the surrogate on a full 256 x 256 film
    (forward and input gradient) against the FP64 oracle on the same
    BF16-rounded operands."""
    H = W = 256
    rng = np.random.default_rng(12)
    params = [(bf16(w).astype(np.float64), bf16(b).astype(np.float64)) for w, b in osg.init_params(2)]
    sur = lib.Surrogate(H, W, max_batch=1)
    sur.set_params(params)
    x = bf16(rng.standard_normal((1, H, W, 32)))
    gy = bf16(rng.standard_normal((1, H, W, 32)))
    y, gx, gw, gb = sur.conv_check(1, x, gy)
    w, b = params[1]
    xo = x[0].transpose(2, 0, 1).astype(np.float64)
    go = gy[0].transpose(2, 0, 1).astype(np.float64)
    y_ref = osg.conv3x3(xo, w, b)
    gx_ref, gw_ref, gb_ref = osg.conv3x3_backward(xo, w, go)
    for got, ref in ((y[0].transpose(2, 0, 1), y_ref), (gx[0].transpose(2, 0, 1), gx_ref), (gw, gw_ref), (gb, gb_ref)):
        e = float(np.max(np.abs(np.asarray(got, np.float64) - ref))) / float(np.max(np.abs(ref)))
        note("256x256 conv layer: rel max", e)
        assert e <= 1e-5
