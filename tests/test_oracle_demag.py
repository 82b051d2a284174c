"""Pins of the oracle's demagnetising tensor and convolution against closed
forms, invariants, brute-force integrals and direct sums (CPU only)."""
import math

import numpy as np
import pytest

from oracle import demag


def _aharoni(a, b, c):
    """Demagnetising factor along the 2c edge of a uniformly magnetised
    rectangular prism 2a x 2b x 2c (A. Aharoni, J. Appl. Phys. 83, 3432
    (1998), Eq. 1)."""
    r = math.sqrt(a * a + b * b + c * c)
    rab, rbc, rac = math.hypot(a, b), math.hypot(b, c), math.hypot(a, c)
    s = ((b * b - c * c) / (2 * b * c) * math.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * math.log((r - b) / (r + b))
         + b / (2 * c) * math.log((rab + a) / (rab - a))
         + a / (2 * c) * math.log((rab + b) / (rab - b))
         + c / (2 * a) * math.log((rbc - b) / (rbc + b))
         + c / (2 * b) * math.log((rac - a) / (rac + a))
         + 2 * math.atan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (rac + rbc)
         - (rab ** 3 + rbc ** 3 + rac ** 3) / (3 * a * b * c))
    return s / math.pi


def _self(dx, dy, dz):
    return demag.cell_tensor(np.array([0]), np.array([0]), np.array([0]), dx, dy, dz)[:, 0]


def test_aharoni_reference_itself():
    # the closed form is only trusted because it reproduces 1/3 for a cube
    # and the trace identity for arbitrary prisms
    assert _aharoni(1, 1, 1) == pytest.approx(1 / 3, abs=1e-14)
    for a, b, c in [(1, 2, 3), (5, 1, 0.1), (2, 2, 0.3)]:
        assert _aharoni(a, b, c) + _aharoni(b, c, a) + _aharoni(c, a, b) == pytest.approx(1, abs=1e-12)


def test_cube_self_term_is_one_third():
    """PIN-1: a cube's self term is 1/3 on the diagonal by symmetry and
    trace 1, with zero off-diagonal terms."""
    N = _self(1.0, 1.0, 1.0)
    np.testing.assert_allclose(N[:3], 1 / 3, atol=1e-14)
    np.testing.assert_allclose(N[3:], 0.0, atol=1e-14)


@pytest.mark.parametrize("cell", [(4e-9, 4e-9, 3e-9), (1.0, 2.0, 5.0), (3.0, 1.0, 0.6)])
def test_self_trace_and_offsite_trace(cell):
    """PIN-2: trace of the self term is 1 for any cuboid (the field of a
    uniformly magnetised body integrates to -M over itself); off-site the
    tensor is traceless (the dipole tensor is)."""
    N = _self(*cell)
    assert N[:3].sum() == pytest.approx(1.0, abs=1e-13)
    rng = np.random.default_rng(0)
    ijk = rng.integers(-12, 13, size=(3, 60))
    ijk = ijk[:, np.any(ijk != 0, axis=0)]
    T = demag.cell_tensor(ijk[0], ijk[1], ijk[2], *cell)
    scale = np.abs(T[:3]).max(axis=0)
    # Newell's 27-point difference cancels (R/d)^6 digits; 1e-7 covers R <= 8 cells
    assert np.all(np.abs(T[:3].sum(axis=0)) <= 1e-7 * scale)


@pytest.mark.parametrize("shape,cell", [((3, 2, 1), (4.0, 4.0, 3.0)),
                                        ((5, 3, 2), (1.0, 1.0, 1.0)),
                                        ((9, 4, 1), (2.0, 1.0, 0.5))])
def test_prism_factors_match_aharoni(shape, cell):
    """PIN-3: the mean field of a uniformly magnetised prism made of cells is
    -Ms D m with D Aharoni's closed form; summing the cell tensor over all
    target/source pairs of the prism gives exactly Ncells * D."""
    n = shape
    geom = {"n": n, "cell": cell, "pbc": (False, False, False)}
    k, j, i = np.meshgrid(range(n[2]), range(n[1]), range(n[0]), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    N = demag.kernel_for_offsets(i[:, None] - i[None, :], j[:, None] - j[None, :],
                                 k[:, None] - k[None, :], geom)
    avg = N.sum(axis=(1, 2)) / len(i)
    a, b, c = (n[q] * cell[q] / 2 for q in range(3))
    np.testing.assert_allclose(avg[:3], [_aharoni(b, c, a), _aharoni(c, a, b), _aharoni(a, b, c)],
                               rtol=1e-9)
    np.testing.assert_allclose(avg[3:], 0.0, atol=1e-12)


def _brute_tensor(i, j, k, cell, nodes=16):
    """The cell-averaged tensor as a brute-force tent-weighted Gauss-Legendre
    integral of the dipole tensor with many nodes; valid where the
    integrand stays away from its singularity (one offset >= 2 cells)."""
    t, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    axes = []
    for d in cell:
        s = np.concatenate([d * t, -d * t])
        ws = np.concatenate([d * w * (d - d * t)] * 2)
        axes.append((s, ws))
    (sx, wx), (sy, wy), (sz, wz) = axes
    SX, SY, SZ = np.meshgrid(sx, sy, sz, indexing="ij")
    W = wx[:, None, None] * wy[None, :, None] * wz[None, None, :]
    G = demag.dipole_tensor(i * cell[0] + SX, j * cell[1] + SY, k * cell[2] + SZ)
    return (G * W).sum(axis=(1, 2, 3)) / (cell[0] * cell[1] * cell[2])


@pytest.mark.parametrize("ijk", [(2, 1, 0), (2, 1, 1), (0, 3, 1), (3, 2, 1), (1, 0, 2), (4, -3, 2)])
def test_newell_matches_brute_force_integral(ijk):
    """PIN-4a: Newell's closed form (every component, including the signs
    of the off-diagonal g terms) equals a brute-force quadrature of the
    defining double volume integral at near offsets."""
    cell = (1.0, 1.2, 0.8)
    newell = demag.newell_tensor(np.array([ijk[0] * cell[0]]), np.array([ijk[1] * cell[1]]),
                                 np.array([ijk[2] * cell[2]]), *cell)[:, 0]
    brute = _brute_tensor(*ijk, cell)
    scale = np.abs(brute).max()
    np.testing.assert_allclose(newell, brute, atol=2e-8 * scale)


def test_far_field_tends_to_point_dipole():
    """PIN-4b: far entries approach V*G(X) with a relative gap falling as
    (d/R)^2."""
    cell = (4.0, 4.0, 3.0)
    V = 48.0
    gaps = []
    for R in (16, 32, 64, 128):
        i, j, k = np.array([R]), np.array([R // 2]), np.array([1])
        N = demag.cell_tensor(i, j, k, *cell)[:, 0]
        G = V * demag.dipole_tensor(i * 4.0, j * 4.0, k * 3.0)[:, 0]
        gaps.append(np.abs(N - G).max() / np.abs(G).max())
    ratios = [gaps[q] / gaps[q + 1] for q in range(3)]
    for r in ratios:
        assert 3.0 < r < 5.0
    assert gaps[-1] < (1.0 / 128) ** 2


def test_near_far_switch_is_continuous():
    """PIN-4c: at the switch distance Newell and the tent quadrature agree to
    about 1e-7 relative (both evaluate the same integral)."""
    cell = (1.0, 1.0, 0.75)
    for ijk in [(8, 0, 0), (8, 3, 1), (0, 8, 2), (5, 8, 0), (8, 8, 0)]:
        X = [np.array([ijk[q] * cell[q]]) for q in range(3)]
        a = demag.newell_tensor(*X, *cell)[:, 0]
        b = demag.far_tensor(*X, *cell)[:, 0]
        assert np.abs(a - b).max() <= 2e-7 * np.abs(a).max()


def test_parity_symmetry_of_tensor():
    """Each component is even or odd under reflection of each offset axis,
    as the cell geometry is symmetric (evaluated directly, not through the
    symmetry shortcut)."""
    cell = (1.0, 1.5, 0.7)
    rng = np.random.default_rng(3)
    for _ in range(10):
        ijk = rng.integers(1, 12, size=3)
        base = demag.cell_tensor(*[np.array([v]) for v in ijk], *cell)[:, 0]
        for flip in range(1, 8):
            s = [(-1 if flip >> q & 1 else 1) for q in range(3)]
            T = demag.cell_tensor(*[np.array([s[q] * ijk[q]]) for q in range(3)], *cell)[:, 0]
            for c, name in enumerate(demag.COMPONENTS):
                p = demag.PARITY[name]
                sign = np.prod([p[q] if s[q] < 0 else 1 for q in range(3)])
                # Newell sums are rounded differently at mirrored offsets
                assert T[c] == pytest.approx(sign * base[c], rel=1e-8, abs=1e-16)


def _rand_m(n, seed):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3, n[2], n[1], n[0]))
    return m / np.linalg.norm(m, axis=0)


@pytest.mark.parametrize("n,pbc", [((5, 3, 2), (False, False, False)),
                                   ((8, 8, 1), (False, False, False)),
                                   ((6, 6, 4), (True, False, False)),
                                   ((6, 5, 3), (True, True, False)),
                                   ((4, 4, 4), (False, True, True))])
def test_fft_convolution_equals_direct_sum(n, pbc):
    """PIN-5: zero-padded FFT convolution equals the direct O(N^2) sum with
    the same kernel (checks padding, wrap-around and the multiply)."""
    geom = {"n": n, "cell": (4e-9, 3.5e-9, 3e-9), "pbc": pbc, "images": 2}
    m = _rand_m(n, sum(n))
    a = demag.demag_field_fft(m, 8e5, geom)
    b = demag.demag_field_direct(m, 8e5, geom)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_direct_sum_far_pairs_are_dipole_sums():
    """Brute-force dipole check: for two cells far apart, the direct sum
    reduces to the field of a point dipole to O((d/R)^2)."""
    n = (40, 1, 1)
    geom = {"n": n, "cell": (2e-9, 2e-9, 2e-9), "pbc": (False,) * 3}
    m = np.zeros((3, 1, 1, 40))
    m[1, 0, 0, 0] = 1.0                     # one cell magnetised along y
    H = demag.demag_field_direct(m, 1e6, geom)
    V = 8e-27
    r = 39 * 2e-9
    # field of a dipole moment Ms V y_hat at distance r along x: -Ms V/(4 pi r^3) y_hat
    expect = -1e6 * V / (4 * math.pi * r ** 3)
    assert H[1, 0, 0, 39] == pytest.approx(expect, rel=1e-3)
    assert abs(H[0, 0, 0, 39]) < 1e-9 * abs(expect)


@pytest.mark.parametrize("n,pbc", [((8, 6, 1), (False, False, False)),
                                   ((7, 6, 3), (True, True, False)),
                                   ((6, 8, 4), (True, False, True)),
                                   ((5, 5, 2), (True, True, True))])
def test_kernel_spectrum_is_real(n, pbc):
    """PIN-16: the symmetric kernel's FP64 transform is real to 1e-12 (this
    also checks the index mapping and the Nyquist averaging)."""
    geom = {"n": n, "cell": (4e-9, 4e-9, 3e-9), "pbc": pbc, "images": 2}
    _, resid = demag.kernel_spectrum(geom)
    assert resid <= 1e-12


def test_periodic_film_limits():
    """PIN-15: an infinite thin film (periodic in x and y) has N_zz = 1 and
    N_xx = N_yy = 0; with finitely many images the residual falls as the
    image count grows."""
    errs = []
    for P in (2, 5, 10):
        geom = {"n": (16, 16, 1), "cell": (4e-9, 4e-9, 3e-9), "pbc": (True, True, False), "images": P}
        mz = np.zeros((3, 1, 16, 16)); mz[2] = 1.0
        mx = np.zeros((3, 1, 16, 16)); mx[0] = 1.0
        hz = demag.demag_field_fft(mz, 1.0, geom)
        hx = demag.demag_field_fft(mx, 1.0, geom)
        errs.append((abs(hz[2].mean() + 1.0), abs(hx[0].mean())))
    assert errs[-1][0] < 5e-3 and errs[-1][1] < 5e-3
    assert errs[0][0] > errs[1][0] > errs[2][0]
    assert errs[0][1] > errs[1][1] > errs[2][1]
