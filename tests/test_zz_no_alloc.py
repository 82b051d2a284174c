"""The no-allocation evaluation (llg_eval_heff_noalloc) against the ordinary
one (llg_eval_heff), through the C ABI: two calls in a row on one GPU, the
second on a smaller film, each equal bit for bit to llg_eval_heff of the same
m on the same solver, and within 1e-5 of the FP64 oracle."""
import numpy as np
import pytest

import workloads
from oracle import fields

pytestmark = pytest.mark.gpu


def maxrel(a, b):
    d = np.linalg.norm((a - b).reshape(3, -1), axis=0).max()
    return d / np.linalg.norm(b.reshape(3, -1), axis=0).max()


def one_film(lib, torch, n, seed, **kw):
    prob, m0 = workloads.small_problem(n, seed=seed, alpha=0.3, **kw)
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    h_ref = s.eval_heff()            # also builds the kernel spectrum (allocates)
    m_dev = torch.from_numpy(s.get_m()).to("cuda:0")
    h_dev = torch.full_like(m_dev, float("nan"))
    torch.cuda.synchronize()
    s.eval_heff_noalloc(m_dev, h_dev)
    h = h_dev.cpu().numpy()
    assert np.array_equal(h, h_ref), f"{n}: differs from llg_eval_heff"
    # the solver's own state is untouched: its evaluation is unchanged
    assert np.array_equal(s.eval_heff(), h_ref)
    e = maxrel(h, fields.heff(s.get_m().astype(np.float64), prob))
    print(f"no-alloc eval {n}: max-rel vs oracle {e:.2e}", flush=True)
    assert e <= 1e-5
    s.close()


def test_noalloc_eval_two_calls(lib):
    import torch
    one_film(lib, torch, (96, 80, 1), seed=21)
    one_film(lib, torch, (40, 24, 1), seed=22)     # smaller: stale scratch from the first call


def test_noalloc_eval_3d_and_rejects(lib):
    import torch
    one_film(lib, torch, (24, 16, 8), seed=23)
    prob, m0 = workloads.small_problem((16, 16, 1), seed=24, alpha=0.3)
    s = lib.Solver(0)
    s.set_problem(prob)
    s.set_m(m0)
    m_dev = torch.from_numpy(m0).to("cuda:0")
    h_dev = torch.empty_like(m_dev)
    with pytest.raises(lib.LLGError) as ei:          # kernel spectrum not built yet
        s.eval_heff_noalloc(m_dev, h_dev)
    assert ei.value.code == lib.LLG_E_STATE
    s.close()
    # a 128 x 128 x 32 block: 14 MB of x spectrum plus 28 MB of y-transformed
    # spectrum, above the 32 MiB static array
    big_prob, big_m = workloads.small_problem((128, 128, 32), seed=25, alpha=0.3)
    big = lib.Solver(0)
    big.set_problem(big_prob)
    big.set_m(big_m)
    big.eval_heff()
    m_dev = torch.from_numpy(big_m).to("cuda:0")
    h_dev = torch.empty_like(m_dev)
    with pytest.raises(lib.LLGError) as ei:
        big.eval_heff_noalloc(m_dev, h_dev)
    assert ei.value.code == lib.LLG_E_UNSUPPORTED
    big.close()
