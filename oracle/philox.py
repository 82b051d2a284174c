"""Philox4x32-10 counter-based generator and the Gaussian draw used for the
thermal field.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 6 of the paper needs Gaussian numbers with zero mean and unit variance,
uncorrelated in space and time; the paper does not say how they are drawn.
Both the oracle and the GPU library implement the same published generator,
Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), each from that definition:

    round:  (hi0, lo0) = M0 * x0,  (hi1, lo1) = M1 * x2   (32x32 -> 64 bit)
            x' = (hi1 ^ x1 ^ k0,  lo1,  hi0 ^ x3 ^ k1,  lo0)
    key schedule: k0 += W0, k1 += W1 between rounds.

Counter and key of the thermal draw for cell c (linear index
i + nx*(j + ny*k)) at step s with a 64-bit seed:

    key = (seed & 0xffffffff, seed >> 32)
    ctr = (c, s & 0xffffffff, s >> 32, 0)

Each 32-bit output x maps to a uniform u = ((x >> 8) + 0.5) * 2^-24 in (0, 1)
(exactly representable in single precision, so both sides see the same u),
and Box-Muller gives eta_x = sqrt(-2 ln u0) cos(2 pi u1),
eta_y = sqrt(-2 ln u0) sin(2 pi u1), eta_z = sqrt(-2 ln u2) cos(2 pi u3).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: sequence of four uint32 arrays (broadcastable); key: two ints.
    Returns four uint32 arrays."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr)
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                          hi0 ^ x3 ^ np.uint64(k1), lo0)
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def uniforms(bits):
    """24-bit uniform in (0, 1) from a uint32."""
    return ((np.asarray(bits, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24


def thermal_eta(ncells, step, seed):
    """Unit Gaussian vectors eta, shape (3, ncells), for one time step."""
    c = np.arange(ncells, dtype=np.uint64)
    s = int(step)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    ctr = (c, np.full_like(c, s & 0xFFFFFFFF), np.full_like(c, (s >> 32) & 0xFFFFFFFF),
           np.zeros_like(c))
    r0, r1, r2, r3 = philox4x32_10(ctr, key)
    u0, u1, u2, u3 = uniforms(r0), uniforms(r1), uniforms(r2), uniforms(r3)
    a = np.sqrt(-2.0 * np.log(u0))
    b = np.sqrt(-2.0 * np.log(u2))
    return np.stack([a * np.cos(2.0 * np.pi * u1),
                     a * np.sin(2.0 * np.pi * u1),
                     b * np.cos(2.0 * np.pi * u3)])
