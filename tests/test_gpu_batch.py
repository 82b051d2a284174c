"""Batched films (one grouped launch per pass over all films): each film's
result equals the single-film solver's bit for bit, does not depend on the
order of films in the batch, and matches the FP64 oracle."""
import numpy as np
import pytest

import workloads
from oracle import llg as ollg

pytestmark = pytest.mark.gpu


def sweep(sides, seed):
    rng = np.random.default_rng(seed)
    films = []
    for side in sides:
        n = (side, side, 1)
        prob = dict(n=n, cell=(4e-9, 4e-9, 3e-9), pbc=(False, False, False),
                    Ms=float(rng.uniform(6e5, 1.2e6)), Aex=1.3e-11, alpha=float(rng.uniform(0.2, 0.5)),
                    Ku=float(rng.uniform(0, 5e3)), u=(1.0, 0.0, 0.0),
                    B=workloads.field_in_plane(float(rng.uniform(0, 0.1)), float(rng.uniform(0, 360))),
                    T=0.0, seed=0)
        films.append((prob, workloads.random_unit(n, int(rng.integers(1 << 30)))))
    return films


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(3, -1)
    b = np.asarray(b, dtype=np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


def test_batch_equals_single_films_bitwise(lib):
    films = sweep((32, 64, 96, 128, 64), 11)
    b = lib.Batch(films)
    st = b.run(4e-12, 1e-5, 1e-14)
    assert all(s["done"] == 1 for s in st)
    for i, (prob, m0) in enumerate(films):
        s = lib.Solver(0)
        s.set_problem(prob)
        s.set_m(m0)
        ss = s.run(4e-12, 1e-5, 1e-14)
        assert b.attempts(i) == s.attempts()
        assert np.array_equal(b.get_m(i), s.get_m())
        assert st[i]["evals"] == ss["evals"] and st[i]["steps"] == ss["steps"]
        print("film", i, prob["n"], "attempts", len(s.attempts()), "identical", flush=True)


def test_batch_order_does_not_matter(lib):
    films = sweep((32, 96, 64), 5)
    a = lib.Batch(films)
    a.run(3e-12, 1e-5, 1e-14)
    perm = [2, 0, 1]
    b = lib.Batch([films[p] for p in perm])
    b.run(3e-12, 1e-5, 1e-14)
    for j, p in enumerate(perm):
        assert np.array_equal(b.get_m(j), a.get_m(p))


def test_batch_film_matches_oracle(lib):
    films = sweep((64, 32), 21)
    b = lib.Batch(films)
    b.run(3e-12, 1e-5, 1e-14)
    for i, (prob, m0) in enumerate(films):
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in b.attempts(i)])
        e = maxrel(b.get_m(i), o.m)
        print("batch film", i, "m maxrel vs oracle", e, flush=True)
        assert e <= 1e-5


def test_batch_rejects_sizes_beyond_the_compiled_lengths(lib):
    prob, m0 = workloads.small_problem(n=(2100, 4, 1))     # x padded beyond 4096
    with pytest.raises(lib.LLGError) as e:
        lib.Batch([(prob, m0)])
    assert e.value.code == lib.LLG_E_UNSUPPORTED


def test_batch_ragged_sizes_match_oracle(lib):
    """Films whose 2n is no compiled length are padded further (17 x 9 to
    64 x 64, 40 x 8 to 128 x 64, 1100 x 4 to 4096 x 64, ...); the
    convolution is unchanged, so each film still follows the oracle, which
    replays its attempts, to 1e-5."""
    films = []
    for n, seed in [((17, 9, 1), 1), ((40, 8, 1), 2), ((150, 30, 1), 3), ((1100, 4, 1), 4)]:
        prob, m0 = workloads.small_problem(n=n, seed=seed, alpha=0.5)
        films.append((prob, m0))
    b = lib.Batch(films)
    st = b.run(2e-12, 1e-5, 1e-14)
    assert all(s["done"] == 1 for s in st)
    for i, (prob, m0) in enumerate(films):
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in b.attempts(i)])
        e = maxrel(b.get_m(i), o.m)
        print("ragged film", prob["n"], "attempts", len(b.attempts(i)), "m maxrel vs oracle", e, flush=True)
        assert e <= 1e-5


def test_sp2_shaped_films_match_oracle(lib):
    """Four films of the relaxation sweep (d/l_ex = 1, 10.7, 20.3, 30; alpha
    = 1, demag and exchange only, from [1,1,1]): 5 ps in one batch, each
    film replayed by the oracle to 1e-5."""
    films, run = workloads.sp2_films(count=4)
    b = lib.Batch(films)
    st = b.run(5e-12, run["tol"], run["dt0"])
    assert all(s["done"] == 1 for s in st)
    for i, (prob, m0) in enumerate(films):
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in b.attempts(i)])
        e = maxrel(b.get_m(i), o.m)
        print("sp2 film d/lex", round(prob["d_over_lex"], 2), prob["n"], "attempts", len(b.attempts(i)),
              "m maxrel vs oracle", e, flush=True)
        assert e <= 1e-5


def test_batch_continues_with_each_films_step(lib):
    """Stopping after 5 attempts and continuing with dt0 = 0 (each film's own
    next step) equals the uninterrupted run bit for bit."""
    films = sweep((32, 64, 96), 9)
    a = lib.Batch(films)
    a.run(3e-12, 1e-5, 1e-14)
    b = lib.Batch(films)
    b.run(3e-12, 1e-5, 1e-14, max_attempts=5)
    b.run(3e-12, 1e-5, 0.0)
    for i in range(len(films)):
        assert b.attempts(i) == a.attempts(i)
        assert np.array_equal(b.get_m(i), a.get_m(i))


def test_full_sweep_creates_and_steps(lib):
    """The 64-film sweep of uneven sizes (sides 64..256) in one batch."""
    films, run = workloads.film_batch()
    b = lib.Batch(films)
    st = b.run(run["t_end"], run["tol"], run["dt0"], max_attempts=4)
    assert all(s["health"] == 0 for s in st)
    assert all(s["evals"] == 1 + 6 * 4 for s in st)



def test_batch_autotune(lib, default_variants):
    """The batch's own autotuner times both compiled variants of every length
    its films use, keeps the faster in the shared table and leaves every
    film's state as it was.  Batches and solvers built afterwards read the
    tuned table: a film of a new batch still equals its single-film run bit
    for bit, and stays within FP32 rounding of the untuned result."""
    films = sweep((32, 64, 96), 21)
    b = lib.Batch(films)
    ref = b.run(1e-12, 1e-5, 1e-14)
    untuned = [b.get_m(i) for i in range(len(films))]
    ent = b.autotune(3)
    print(ent, flush=True)
    assert sorted((e["kind"], e["length"]) for e in ent) == \
        sorted([("row", 64), ("row", 128), ("row", 192), ("col", 32), ("col", 64), ("col", 96)])
    for e in ent:
        usable = [v for v in (0, 1) if e["ms"][v] >= 0]
        assert usable and all(e["ms"][v] > 0 for v in usable)
        assert e["variant"] == min(usable, key=lambda v: e["ms"][v])
    for i in range(len(films)):
        assert np.array_equal(b.get_m(i), untuned[i])
    assert [s["steps"] for s in b.run(1e-12, 1e-5, 0.0)] == [s["steps"] for s in ref]   # already there
    t = lib.Batch(films)
    st = t.run(1e-12, 1e-5, 1e-14)
    for i, (prob, m0) in enumerate(films):
        s = lib.Solver(0)
        s.set_problem(prob)
        s.set_m(m0)
        s.run(1e-12, 1e-5, 1e-14)
        assert np.array_equal(t.get_m(i), s.get_m())
        assert st[i]["done"] == 1
        assert maxrel(t.get_m(i), untuned[i]) <= 1e-4


# films whose padded row lengths have a four-class variant 1 (128, 256, 384,
# 512), two of them square with the single-film padding, three ragged
# (nx < Px / 2, ny < L)
FORCED = [((64, 64, 1), 31), ((128, 96, 1), 32), ((150, 30, 1), 33), ((100, 50, 1), 34), ((200, 20, 1), 35)]


def test_forced_variants_advance_and_match(lib, default_variants):
    """A batch whose row lengths are switched from two to four frequency
    classes (and a column length to its other variant) after creation is
    advanced itself: every film follows the FP64 oracle, which replays its
    attempts, to 1e-5, and the square films equal single-film solvers on
    the same variants bit for bit.  (Launch arguments built for the old row
    variant would read the spectrum in the wrong column order.)"""
    films = [workloads.small_problem(n=n, seed=seed, alpha=0.3) for n, seed in FORCED]
    b = lib.Batch(films)
    for px in (128, 256, 384, 512):
        b.set_variant("row", px, 1)
    b.set_variant("col", 64, 1)
    with pytest.raises(lib.LLGError) as e:
        b.set_variant("row", 640, 1)
    assert e.value.code == lib.LLG_E_ARG
    st = b.run(2e-12, 1e-5, 1e-14)
    assert all(s["done"] == 1 for s in st)
    for i, (prob, m0) in enumerate(films):
        o = ollg.Solver(prob, m0)
        o.replay([(dt, ok) for dt, _, ok in b.attempts(i)])
        e = maxrel(b.get_m(i), o.m)
        print("forced-variant film", prob["n"], "attempts", len(b.attempts(i)), "m maxrel vs oracle", e, flush=True)
        assert e <= 1e-5
    for i, rv, cv in ((0, 1, 1), (1, 1, 0)):
        prob, m0 = films[i]
        s = lib.Solver(0)
        s.set_problem(prob)
        s.set_variants(rv, cv)
        s.set_m(m0)
        s.run(2e-12, 1e-5, 1e-14)
        assert b.attempts(i) == s.attempts()
        assert np.array_equal(b.get_m(i), s.get_m()), f"film {i}"


def test_batch_autotune_then_advance(lib, default_variants):
    """The tuned batch object itself keeps integrating correctly: after
    llg_batch_autotune it is advanced and replayed by the oracle (1e-5),
    also when the tuner kept four-class rows."""
    films = [workloads.small_problem(n=n, seed=seed, alpha=0.3) for n, seed in FORCED]
    b = lib.Batch(films)
    b.run(1e-12, 1e-5, 1e-14)
    mid = [b.get_m(i) for i in range(len(films))]
    seen = [len(b.attempts(i)) for i in range(len(films))]
    ent = b.autotune(2)
    print("tuned", ent, flush=True)
    st = b.run(3e-12, 1e-5, 0.0)
    assert all(s["done"] == 1 for s in st)
    for i, (prob, _) in enumerate(films):
        o = ollg.Solver(prob, mid[i])
        o.replay([(dt, ok) for dt, _, ok in b.attempts(i)[seen[i]:]])
        e = maxrel(b.get_m(i), o.m)
        print("tuned film", prob["n"], "m maxrel vs oracle", e, flush=True)
        assert e <= 1e-5
    # the same with the tuner's choices forced the other way round
    for x in ent:
        if x["ms"][1 - x["variant"]] >= 0:
            b.set_variant(x["kind"], x["length"], 1 - x["variant"])
    mid = [b.get_m(i) for i in range(len(films))]
    seen = [len(b.attempts(i)) for i in range(len(films))]
    b.run(5e-12, 1e-5, 0.0)
    for i, (prob, _) in enumerate(films):
        o = ollg.Solver(prob, mid[i])
        o.replay([(dt, ok) for dt, _, ok in b.attempts(i)[seen[i]:]])
        e = maxrel(b.get_m(i), o.m)
        print("flipped film", prob["n"], "m maxrel vs oracle", e, flush=True)
        assert e <= 1e-5
