"""The longest compiled transforms: 4096-point rows (films 2026 ... 2048
cells wide, or 4096 periodic) and columns of half length 2048 (films 2026
... 2048 cells tall), whose kernels read the magnetisation from global
memory and share the FFT scratch with the exchange (Sec. 3.2 stages i-iii).
Every variant against the FP64 oracle: H_eff, then adaptive Dormand-Prince
attempts replayed by the oracle; the full 2048 x 2048 film against stored
oracle values at sampled cells."""
import os

import numpy as np
import pytest

import workloads
from oracle import fields, llg as ollg

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def note(*a):
    print(*a, flush=True)


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(3, -1)
    b = np.asarray(b, dtype=np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


def solver(lib, prob, m0):
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    return s


@pytest.mark.parametrize("n,pbc", [((2048, 32, 1), (False, False, False)),
                                   ((2039, 32, 1), (False, False, False)),
                                   ((4096, 32, 1), (True, False, False)),
                                   ((32, 2048, 1), (False, False, False)),
                                   ((32, 2030, 1), (False, False, False))])
def test_long_transforms_every_variant(lib, default_variants, n, pbc):
    """H_eff of every (row, column) variant pair, then three adaptive
    Dormand-Prince attempts of each row (or column) variant replayed by the
    oracle; ragged films included."""
    prob, m0 = workloads.small_problem(n, pbc=pbc, seed=n[0] + 3 * n[1], alpha=0.3)
    note("case:", n, "pbc", pbc)
    ref = fields.heff(m0.astype(np.float64), prob)
    s = solver(lib, prob, m0)
    for rv in range(2):
        for cv in range(2):
            s.set_variants(rv, cv)
            e = maxrel(s.eval_heff(), ref)
            note("  variants", (rv, cv), "H_eff maxrel", e)
            assert e <= 1e-5
    for v in range(2):
        s.set_variants(v, v)
        s.set_m(m0)
        st = s.run_attempts(5e-12, 1e-5, 1e-14, 3)
        log = s.attempts()
        assert len(log) == 3 and st["evals"] == 1 + 6 * 3
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in log])
        e = maxrel(s.get_m(), o.m)
        note("  dp45 variants", (v, v), "m maxrel", e)
        assert e <= 1e-5


def test_film_2048_sampled(lib, default_variants):
    """The 2048 x 2048 film (FFT grid 4096 x 4096) with every variant pair:
    H_eff at 4096 cells against the oracle values stored by
    tests/golden/make_film2048_samples.py (the oracle's whole-film FP64
    convolution takes minutes, so it is not rerun here)."""
    path = os.path.join(HERE, "golden", "film2048_heff_samples.txt")
    data = np.loadtxt(path)
    idx = data[:, 0].astype(np.int64)
    ref = data[:, 1:].T
    prob, m0 = workloads.small_problem((2048, 2048, 1), seed=2048, alpha=0.3)
    s = solver(lib, prob, m0)
    for rv in range(2):
        for cv in range(2):
            s.set_variants(rv, cv)
            h = s.eval_heff().reshape(3, -1)[:, idx]
            e = maxrel(h, ref)
            note("2048x2048 variants", (rv, cv), "H_eff maxrel at", len(idx), "cells:", e)
            assert e <= 1e-5
