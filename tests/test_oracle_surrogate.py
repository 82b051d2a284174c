"""Pins of the surrogate oracle: the convolution against scipy's direct
correlation and a naive loop, every gradient against central differences,
Adam against its closed form on a quadratic."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import surrogate as sg


def test_conv_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4, 7, 9))
    w = rng.standard_normal((5, 4, 3, 3))
    b = rng.standard_normal(5)
    y = sg.conv3x3(x, w, b)
    for o in range(5):
        ref = b[o] + sum(correlate(x[c], w[o, c], mode="same") for c in range(4))
        np.testing.assert_allclose(y[o], ref, rtol=1e-12, atol=1e-12)


def test_conv_matches_naive_loop():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 5))
    w = rng.standard_normal((3, 2, 3, 3))
    b = np.zeros(3)
    y = sg.conv3x3(x, w, b)
    for o in range(3):
        for i in range(4):
            for j in range(5):
                acc = 0.0
                for c in range(2):
                    for u in range(3):
                        for v in range(3):
                            ii, jj = i + u - 1, j + v - 1
                            if 0 <= ii < 4 and 0 <= jj < 5:
                                acc += w[o, c, u, v] * x[c, ii, jj]
                assert y[o, i, j] == pytest.approx(acc, abs=1e-12)


def _small_params(rng):
    layers = ((3, 4), (4, 4), (4, 2))
    return [(rng.standard_normal((co, ci, 3, 3)) * 0.5, rng.standard_normal(co) * 0.1) for ci, co in layers]


def test_gradients_by_central_differences():
    """PIN-18a: every weight, bias and input gradient of the FP64 backward
    pass agrees with central differences of the loss (<= 1e-6 relative)."""
    rng = np.random.default_rng(2)
    params = _small_params(rng)
    x = rng.standard_normal((3, 5, 6))
    target = rng.standard_normal((2, 5, 6))
    loss, grads = sg.loss_and_grads(params, x, target)
    h = 1e-6
    for li in range(len(params)):
        for k in range(2):
            p = params[li][k]
            g = grads[li][k]
            flat = p.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = sg.loss_and_grads(params, x, target)
                flat[idx] = old - h
                lm, _ = sg.loss_and_grads(params, x, target)
                flat[idx] = old
                num = (lp - lm) / (2 * h)
                assert g.reshape(-1)[idx] == pytest.approx(num, rel=1e-6, abs=1e-9)


def test_adam_on_a_quadratic():
    """Adam's first step moves every parameter by lr * sign(g) (bias
    correction makes m/sqrt(v) = g/|g|), and the iteration converges on a
    convex quadratic."""
    params = [(np.array([[[[3.0]]]]), np.array([-2.0]))]
    state = {}
    grads = [(2 * params[0][0], 2 * params[0][1])]
    new = sg.adam_step(params, grads, state, 0.1, 1)
    np.testing.assert_allclose(new[0][0], 3.0 - 0.1, rtol=1e-7)
    np.testing.assert_allclose(new[0][1], -2.0 + 0.1, rtol=1e-7)
    p = new
    for t in range(2, 400):
        p = sg.adam_step(p, [(2 * p[0][0], 2 * p[0][1])], state, 0.05, t)
    assert abs(p[0][0].item()) < 1e-2 and abs(p[0][1].item()) < 1e-2


def test_proposal_keeps_unit_norm():
    rng = np.random.default_rng(3)
    params = sg.init_params(0)
    m = rng.standard_normal((3, 8, 8))
    m /= np.linalg.norm(m, axis=0)
    mp = sg.propose(params, m, (0.01, 0.0, 0.0))
    np.testing.assert_allclose(np.linalg.norm(mp, axis=0), 1.0, rtol=1e-12)


def test_bf16_rounding_and_split_input():
    """round_bf16 is the nearest BF16 value with ties to even (checked
    against a brute-force search over the neighbouring BF16 values), and the
    input pair (hi, lo) holds m: hi + lo / 256 = m exactly in FP32, |lo| <=
    256 * half a BF16 unit of hi."""
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(0.01, 1, 1000), -rng.uniform(0.01, 1, 1000),
                        [1.0, -1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8]])
    x = x.astype(np.float32)
    r = sg.round_bf16(x)
    assert sg.round_bf16(np.zeros(1, np.float32))[0] == 0.0
    for v, got in zip(x, r):
        u = int(np.array([v], np.float32).view(np.uint32)[0]) & 0xFFFF0000
        cands = [np.array([c], np.uint32).view(np.float32)[0] for c in (u - 0x10000, u, u + 0x10000)]
        d = [abs(float(c) - float(v)) for c in cands]
        best = min(d)
        ties = [c for c, e in zip(cands, d) if e == best]
        want = ties[0] if len(ties) == 1 else [c for c in ties if (np.array([c], np.float32).view(np.uint32)[0] >> 16) % 2 == 0][0]
        assert got == want
    m = rng.standard_normal((3, 5, 7)).astype(np.float32)
    xin = sg.net_input(m, (0.01, 0.02, 0.0))
    hi, lo = xin[:3].astype(np.float32), xin[3:6].astype(np.float32)
    assert np.array_equal(hi + lo / np.float32(256.0), m)
    assert np.all(np.abs(lo) <= 256 * np.abs(hi) * 2.0 ** -8 + 1e-30)
    assert np.allclose(xin[6:], np.array([0.2, 0.4, 0.0]).reshape(3, 1, 1))
