"""Magnetostatic (demagnetising) field of a finite-difference grid, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (Sec. 2.1.1, Eq. 2) defines the magnetostatic field as the volume
integral of -(1/4pi) grad grad (1/|r-r'|) . M(r') and evaluates it, on the
finite-difference grid of uniformly magnetised cuboid cells, as a discrete
convolution of M with a cell-to-cell kernel, accelerated by zero-padded FFTs
(Sec. 3.2).  The discrete kernel is the cell-averaged tensor

    N(X) = (1/V) int_cell_i int_cell_j  -(1/4pi) grad grad (1/|r - r'|) dr' dr,
    H_d(r_i) = -Ms * sum_j N(r_i - r_j) . m_j,

with X = r_i - r_j.  The paper does not print a formula for N; this oracle
reads it as follows:

* offsets within NEAR_CELLS cells (max-norm, in cells): the closed form of
  Newell, Williams & Dunlop (J. Geophys. Res. 98, 9551, 1993), a signed
  27-point second difference of the functions f (diagonal) and g
  (off-diagonal);
* farther offsets: the same integral written as the point-dipole tensor G
  averaged against the product of per-axis tent functions (the
  autocorrelation of the box), evaluated by 3-point Gauss-Legendre on each
  half of each axis (216 nodes);
* periodic directions (Sec. 2.1.1): the kernel is the sum of the central
  cell tensor and point-dipole images V*G(X + n L), n = -P..P per periodic
  axis, n != 0; at the Nyquist offset N/2 of an even periodic length the two
  representatives +N/2 and -N/2 are averaged so that the kernel stays
  symmetric (its Fourier transform then is real, Sec. 3.2).

Two evaluations of the field are provided: the zero-padded FFT convolution
of Sec. 3.2 (numpy's FP64 FFT as the library primitive) and the direct
O(N^2) sum, which serves as its check.
"""
import math
from functools import lru_cache

import numpy as np

NEAR_CELLS = 8          # max-norm distance (in cells) up to which Newell is used
DEFAULT_IMAGES = 10     # periodic images per periodic axis

# component order used throughout: xx, yy, zz, xy, xz, yz
COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
# parity of each component under reflection of the X, Y, Z offset
# (+1 even, -1 odd); diagonal terms are even in every axis, N_ab is odd in a
# and in b.
PARITY = {
    "xx": (1, 1, 1), "yy": (1, 1, 1), "zz": (1, 1, 1),
    "xy": (-1, -1, 1), "xz": (-1, 1, -1), "yz": (1, -1, -1),
}


# --------------------------------------------------------------------------
# Newell-Williams-Dunlop near field
# --------------------------------------------------------------------------
def newell_f(x, y, z):
    """Newell's f(x, y, z): even in each argument; terms whose prefactor
    vanishes are taken as zero (their limits are zero)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    y = np.abs(np.asarray(y, dtype=np.float64))
    z = np.abs(np.asarray(z, dtype=np.float64))
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2.0 * x2 - y2 - z2) * R / 6.0
    with np.errstate(divide="ignore", invalid="ignore"):
        rxz = np.sqrt(x2 + z2)
        out = out + np.where(rxz > 0, 0.5 * y * (z2 - x2) * np.arcsinh(y / rxz), 0.0)
        rxy = np.sqrt(x2 + y2)
        out = out + np.where(rxy > 0, 0.5 * z * (y2 - x2) * np.arcsinh(z / rxy), 0.0)
        xR = x * R
        out = out - np.where(xR > 0, x * y * z * np.arctan(y * z / xR), 0.0)
    return out


def newell_g(x, y, z):
    """Newell's g(x, y, z): odd in x and in y, even in z."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    sgn = np.sign(x) * np.sign(y)
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = -x * y * R / 3.0
    with np.errstate(divide="ignore", invalid="ignore"):
        rxy = np.sqrt(x2 + y2)
        out = out + np.where(rxy > 0, x * y * z * np.arcsinh(z / rxy), 0.0)
        ryz = np.sqrt(y2 + z2)
        out = out + np.where(ryz > 0, y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(x / ryz), 0.0)
        rxz = np.sqrt(x2 + z2)
        out = out + np.where(rxz > 0, x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(y / rxz), 0.0)
        zR = z * R
        out = out - np.where(zR > 0, z2 * z / 6.0 * np.arctan(x * y / zR), 0.0)
        yR = y * R
        out = out - np.where(yR > 0, z * y2 / 2.0 * np.arctan(x * z / yR), 0.0)
        xR = x * R
        out = out - np.where(xR > 0, z * x2 / 2.0 * np.arctan(y * z / xR), 0.0)
    return sgn * out


_W = ((-1, -1.0), (0, 2.0), (1, -1.0))   # second-difference weights


def _newell_sum(F, X, Y, Z, dx, dy, dz):
    acc = 0.0
    for a, wa in _W:
        for b, wb in _W:
            for c, wc in _W:
                acc = acc + (wa * wb * wc) * F(X + a * dx, Y + b * dy, Z + c * dz)
    return acc / (4.0 * math.pi * dx * dy * dz)


def newell_tensor(X, Y, Z, dx, dy, dz):
    """All six components (xx, yy, zz, xy, xz, yz) of the cell-averaged tensor
    for offsets X, Y, Z (same length unit as dx, dy, dz), by Newell's formulas.
    The yy/zz/xz/yz entries follow from xx/xy by permuting the axes."""
    return np.stack([
        _newell_sum(newell_f, X, Y, Z, dx, dy, dz),
        _newell_sum(newell_f, Y, X, Z, dy, dx, dz),
        _newell_sum(newell_f, Z, Y, X, dz, dy, dx),
        _newell_sum(newell_g, X, Y, Z, dx, dy, dz),
        _newell_sum(newell_g, X, Z, Y, dx, dz, dy),
        _newell_sum(newell_g, Y, Z, X, dy, dz, dx),
    ])


# --------------------------------------------------------------------------
# point dipole and far field
# --------------------------------------------------------------------------
def dipole_tensor(x, y, z):
    """G(r) = (1/4pi)(delta_ab / r^3 - 3 r_a r_b / r^5): the tensor with
    H = -G . (moment) for a point dipole at the origin."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    inv3 = 1.0 / (r2 * r)
    inv5 = inv3 / r2
    c = 1.0 / (4.0 * math.pi)
    return np.stack([
        c * (inv3 - 3.0 * x * x * inv5),
        c * (inv3 - 3.0 * y * y * inv5),
        c * (inv3 - 3.0 * z * z * inv5),
        c * (-3.0 * x * y * inv5),
        c * (-3.0 * x * z * inv5),
        c * (-3.0 * y * z * inv5),
    ])


_GL3_T = (0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6))
_GL3_W = (5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0)


def tent_nodes(d):
    """Nodes and weights integrating a smooth function against the tent
    (d - |s|)^+ on [-d, d]: 3-point Gauss-Legendre on [-d, 0] and [0, d]."""
    nodes, weights = [], []
    for t, w in zip(_GL3_T, _GL3_W):
        for sgn in (1.0, -1.0):
            s = sgn * d * t
            nodes.append(s)
            weights.append(d * w * (d - abs(s)))
    return nodes, weights


def far_tensor(X, Y, Z, dx, dy, dz):
    """Cell-averaged tensor as the tent-weighted average of the point-dipole
    tensor, N(X) = (1/V) int G(X + s) prod_a (d_a - |s_a|)^+ ds."""
    nx_, wx_ = tent_nodes(dx)
    ny_, wy_ = tent_nodes(dy)
    nz_, wz_ = tent_nodes(dz)
    acc = 0.0
    for sx, wx in zip(nx_, wx_):
        for sy, wy in zip(ny_, wy_):
            for sz, wz in zip(nz_, wz_):
                acc = acc + (wx * wy * wz) * dipole_tensor(X + sx, Y + sy, Z + sz)
    return acc / (dx * dy * dz)


def cell_tensor(i, j, k, dx, dy, dz):
    """Tensor between two cells whose centres differ by (i dx, j dy, k dz),
    i, j, k integer arrays: Newell within NEAR_CELLS cells, tent quadrature
    beyond.  Returns an array of shape (6,) + broadcast shape."""
    i, j, k = np.broadcast_arrays(np.asarray(i), np.asarray(j), np.asarray(k))
    # lengths in units of the largest cell edge (the tensor is scale free)
    s = max(dx, dy, dz)
    ex, ey, ez = dx / s, dy / s, dz / s
    out = np.zeros((6,) + i.shape)
    reach = np.maximum(np.maximum(np.abs(i), np.abs(j)), np.abs(k))
    near = reach <= NEAR_CELLS
    if near.any():
        out[:, near] = newell_tensor(i[near] * ex, j[near] * ey, k[near] * ez, ex, ey, ez)
    far = ~near
    if far.any():
        out[:, far] = far_tensor(i[far] * ex, j[far] * ey, k[far] * ez, ex, ey, ez)
    return out


def periodic_tensor(i, j, k, geom):
    """Central cell tensor plus point-dipole periodic images (Sec. 2.1.1)."""
    dx, dy, dz = geom["cell"]
    nxyz = geom["n"]
    pbc = geom["pbc"]
    P = geom.get("images", DEFAULT_IMAGES)
    out = cell_tensor(i, j, k, dx, dy, dz)
    if not any(pbc):
        return out
    rng = [range(-P, P + 1) if pbc[a] else range(0, 1) for a in range(3)]
    V = dx * dy * dz
    i = np.asarray(i, dtype=np.float64)
    j = np.asarray(j, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    for a in rng[0]:
        for b in rng[1]:
            for c in rng[2]:
                if a == 0 and b == 0 and c == 0:
                    continue
                out = out + V * dipole_tensor((i + a * nxyz[0]) * dx,
                                              (j + b * nxyz[1]) * dy,
                                              (k + c * nxyz[2]) * dz)
    return out


def axis_representatives(d, n, periodic):
    """Offsets (in cells) and weights that a signed offset d along one axis
    stands for.  Open axis: d itself.  Periodic axis of length n: d reduced
    modulo n to the minimal image; the Nyquist offset n/2 of an even n
    stands for +n/2 and -n/2 with weight 1/2 each.  Returns a list of
    (offsets, weights) array pairs."""
    d = np.asarray(d)
    if not periodic:
        return [(d, np.ones(d.shape))]
    r = np.mod(d, n)
    r = np.where(r > n // 2, r - n, r)
    if n % 2:
        return [(r, np.ones(d.shape))]
    nyq = r == n // 2
    return [(r, np.where(nyq, 0.5, 1.0)), (np.full(d.shape, -(n // 2)), np.where(nyq, 0.5, 0.0))]


def _tensor_by_symmetry(i, j, k, geom):
    """periodic_tensor on integer offsets, evaluated once per distinct
    |offset| triple; the sign of each component under reflection of an axis
    is its parity (PARITY), which is a symmetry of the cell geometry and of
    the symmetric image set."""
    A = np.stack([np.abs(i), np.abs(j), np.abs(k)], axis=1)
    uniq, inv = np.unique(A, axis=0, return_inverse=True)
    inv = inv.ravel()
    vals = periodic_tensor(uniq[:, 0], uniq[:, 1], uniq[:, 2], geom)[:, inv]
    sx, sy, sz = np.sign(i), np.sign(j), np.sign(k)
    for c, name in enumerate(COMPONENTS):
        px, py, pz = PARITY[name]
        s = np.ones(i.shape)
        if px < 0:
            s = s * sx
        if py < 0:
            s = s * sy
        if pz < 0:
            s = s * sz
        vals[c] = vals[c] * s
    return vals


def kernel_for_offsets(di, dj, dk, geom):
    """Kernel entries for integer offset arrays (target minus source cell),
    applying the periodic representative rule per axis."""
    di, dj, dk = np.broadcast_arrays(np.asarray(di), np.asarray(dj), np.asarray(dk))
    shape = di.shape
    di, dj, dk = di.ravel(), dj.ravel(), dk.ravel()
    nxyz = geom["n"]
    pbc = geom["pbc"]
    out = np.zeros((6, di.size))
    for a, wa in axis_representatives(di, nxyz[0], pbc[0]):
        for b, wb in axis_representatives(dj, nxyz[1], pbc[1]):
            for c, wc in axis_representatives(dk, nxyz[2], pbc[2]):
                w = wa * wb * wc
                sel = w > 0
                if not sel.any():
                    continue
                out[:, sel] += w[sel] * _tensor_by_symmetry(a[sel], b[sel], c[sel], geom)
    return out.reshape((6,) + shape)


# --------------------------------------------------------------------------
# the convolution kernel on the FFT grid
# --------------------------------------------------------------------------
def fft_lengths(geom):
    """Zero padding (Sec. 3.2): 2N along open axes, N along periodic ones."""
    return tuple(n if p else (2 * n if n > 1 else 1) for n, p in zip(geom["n"], geom["pbc"]))


def _axis_offsets(n, P, periodic):
    """Signed offset represented by each FFT index along one axis, or None
    for the indices that only ever multiply padding zeros."""
    offs = []
    for idx in range(P):
        if periodic:
            offs.append(idx)                        # reduced by axis_representatives
        elif idx < n:
            offs.append(idx)
        elif idx > P - n:
            offs.append(idx - P)
        else:
            offs.append(None)
    return offs


@lru_cache(maxsize=8)
def _kernel_grid_cached(key):
    geom = _geom_from_key(key)
    nx, ny, nz = geom["n"]
    Px, Py, Pz = fft_lengths(geom)
    ox = _axis_offsets(nx, Px, geom["pbc"][0])
    oy = _axis_offsets(ny, Py, geom["pbc"][1])
    oz = _axis_offsets(nz, Pz, geom["pbc"][2])
    grid = np.zeros((6, Pz, Py, Px))
    vx = [q for q, o in enumerate(ox) if o is not None]
    vy = [q for q, o in enumerate(oy) if o is not None]
    vz = [q for q, o in enumerate(oz) if o is not None]
    Ox = np.array([ox[q] for q in vx])
    Oy = np.array([oy[q] for q in vy])
    Oz = np.array([oz[q] for q in vz])
    KZ, KY, KX = np.meshgrid(Oz, Oy, Ox, indexing="ij")
    vals = kernel_for_offsets(KX, KY, KZ, geom)
    grid[np.ix_(range(6), vz, vy, vx)] = vals
    return grid


def _geom_key(geom):
    return (tuple(geom["n"]), tuple(float(c) for c in geom["cell"]),
            tuple(bool(p) for p in geom["pbc"]), int(geom.get("images", DEFAULT_IMAGES)))


def _geom_from_key(key):
    n, cell, pbc, images = key
    return {"n": n, "cell": cell, "pbc": pbc, "images": images}


def kernel_grid(geom):
    """Real-space kernel N on the (Pz, Py, Px) FFT grid, components first.
    Index q along an open axis of length P holds offset q (q < n) or q - P
    (q > P - n); other indices are zero.  Along a periodic axis every index
    is the minimal-image offset."""
    return _kernel_grid_cached(_geom_key(geom))


def kernel_spectrum(geom):
    """FP64 Fourier transform of the kernel.  The kernel is symmetric (each
    component even or odd in every axis), so the transform is real up to
    rounding (Sec. 3.2); returns (real part, max |imag| / max |real|)."""
    grid = kernel_grid(geom)
    spec = np.fft.fftn(grid, axes=(1, 2, 3))
    scale = np.max(np.abs(spec.real))
    resid = float(np.max(np.abs(spec.imag)) / scale) if scale > 0 else 0.0
    return spec.real, resid


def demag_field_fft(m, Ms, geom):
    """H_d = -Ms N * m by zero-padded FFT convolution (Sec. 3.2, stages
    (i)-(iii)).  m has shape (3, nz, ny, nx); returns A/m, same shape."""
    nx, ny, nz = geom["n"]
    P = fft_lengths(geom)
    Khat, _ = kernel_spectrum(geom)
    Mpad = np.zeros((3, P[2], P[1], P[0]))
    Mpad[:, :nz, :ny, :nx] = Ms * np.asarray(m, dtype=np.float64)
    Mhat = np.fft.fftn(Mpad, axes=(1, 2, 3))
    xx, yy, zz, xy, xz, yz = Khat
    Hhat = -np.stack([
        xx * Mhat[0] + xy * Mhat[1] + xz * Mhat[2],
        xy * Mhat[0] + yy * Mhat[1] + yz * Mhat[2],
        xz * Mhat[0] + yz * Mhat[1] + zz * Mhat[2],
    ])
    H = np.fft.ifftn(Hhat, axes=(1, 2, 3)).real
    return H[:, :nz, :ny, :nx].copy()


def demag_field_direct(m, Ms, geom):
    """H_d by the direct O(N^2) sum over all source cells (tiny grids)."""
    nx, ny, nz = geom["n"]
    m = np.asarray(m, dtype=np.float64).reshape(3, -1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    di = i[:, None] - i[None, :]
    dj = j[:, None] - j[None, :]
    dk = k[:, None] - k[None, :]
    N = kernel_for_offsets(di, dj, dk, geom)          # (6, ntarget, nsource)
    xx, yy, zz, xy, xz, yz = N
    H = -Ms * np.stack([
        (xx * m[0] + xy * m[1] + xz * m[2]).sum(axis=1),
        (xy * m[0] + yy * m[1] + yz * m[2]).sum(axis=1),
        (xz * m[0] + yz * m[1] + zz * m[2]).sum(axis=1),
    ])
    return H.reshape(3, nz, ny, nx)
