"""Writes film2048_heff_samples.txt: the FP64 oracle's effective field (all
terms of Sec. 2.1: demag by Eq. 2 as a zero-padded FFT convolution, exchange
Eq. 3, uniaxial anisotropy Eq. 4, Zeeman) of a random 2048 x 2048 x 1 film at
4096 sampled cells, for the full-size check of the 4096-point row and
2048-half-length column kernels.  Calls only oracle/ (and the seeded input
generator); takes a few minutes and ~7 GB.

    python3 tests/golden/make_film2048_samples.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import fields  # noqa: E402

N = 2048
SEED = 2048
NSAMPLE = 4096


def problem():
    return workloads.small_problem((N, N, 1), seed=SEED, alpha=0.3)


def sample_cells():
    """Flat cell indices: the four corners and the edge midpoints, then
    random cells (seeded)."""
    fixed = [0, N - 1, (N - 1) * N, N * N - 1, N // 2, (N // 2) * N, (N // 2) * N + N - 1, (N - 1) * N + N // 2]
    rng = np.random.default_rng(SEED + 1)
    rnd = rng.choice(N * N, size=NSAMPLE - len(fixed), replace=False)
    return np.concatenate([np.array(fixed, dtype=np.int64), rnd.astype(np.int64)])


def main():
    prob, m0 = problem()
    h = fields.heff(m0.astype(np.float64), prob).reshape(3, -1)
    idx = sample_cells()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "film2048_heff_samples.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle H_eff (A/m) of workloads.small_problem((2048, 2048, 1), seed=2048, alpha=0.3)\n")
        f.write("# at sampled cells; columns: flat cell index, Hx, Hy, Hz\n")
        f.write("# written by tests/golden/make_film2048_samples.py (oracle only)\n")
        for i in idx:
            f.write(f"{int(i)} {h[0, i]:.17e} {h[1, i]:.17e} {h[2, i]:.17e}\n")
    print("wrote", out, len(idx), "cells")


if __name__ == "__main__":
    main()
