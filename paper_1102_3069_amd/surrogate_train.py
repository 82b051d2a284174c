"""Data generation and training loop of the learned surrogate.

Orchestration only: the trajectories come from the library's batched fixed
RK4 steps, every loss, gradient and Adam update from its MFMA training
kernels (``Surrogate.train_step``).  Python picks minibatches (index copies
of device tensors) and the learning rate; it does no arithmetic of the
method or of the network.
"""
import math
import time

import numpy as np


def generate_pairs(lib, films, run, pairs_per_traj, predictor="rk4"):
    """Integrates every film of `films` (list of (problem, m0)) together with
    fixed RK4 steps and records its state every `seg_steps` steps after the
    burn-in.  Returns (X, E, B): X a CUDA tensor (ntraj, pairs + 1, 3, H, W),
    consecutive entries one segment apart; E (ntraj, pairs, 3, H, W) the
    plain solver's single coarse step ("rk4" or "euler") over the whole
    segment from each X[:, k] (the proposal base), or None for predictor
    None; B (ntraj, 3) float32 tesla."""
    import torch
    ntraj = len(films)
    nx, ny, _ = films[0][0]["n"]
    b = lib.Batch(films)
    eb = lib.Batch(films) if predictor else None
    if run["burn_in"]:
        b.step(run["method"], run["dt"], run["burn_in"])
    X = torch.empty((ntraj, pairs_per_traj + 1, 3, ny, nx), device="cuda", dtype=torch.float32)
    E = torch.empty((ntraj, pairs_per_traj, 3, ny, nx), device="cuda", dtype=torch.float32) if predictor else None
    for k in range(pairs_per_traj + 1):
        for i in range(ntraj):
            b.get_m(i, out=X[i, k])
        if k < pairs_per_traj:
            if predictor:
                for i in range(ntraj):
                    eb.set_m(i, X[i, k])
                eb.step(predictor, run["dt"] * run["seg_steps"], 1)
                for i in range(ntraj):
                    eb.get_m(i, out=E[i, k])
            b.step(run["method"], run["dt"], run["seg_steps"])
    torch.cuda.synchronize()
    b.close()
    if eb is not None:
        eb.close()
    B = np.array([f[0]["B"] for f in films], dtype=np.float32)
    return X, E, B


def cosine_lr(step, total, lr0, lr_min=0.0):
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * min(step, total) / total))


def train(sur, X, B, steps, batch, lr0=1e-3, seed=0, log_every=0, log=print, E=None):
    """Adam on random minibatches of pairs (X[i, k], X[i, k + 1]), with the
    proposal bases E[i, k] when given, under a cosine learning-rate decay.
    Returns a dict with the loss history and the throughput in pixels per
    second (pixels x samples / wall time)."""
    import torch
    rng = np.random.default_rng(seed)
    ntraj, npairs = X.shape[0], X.shape[1] - 1
    H, W = X.shape[-2:]
    m_in = torch.empty((batch, 3, H, W), device="cuda", dtype=torch.float32)
    m_t = torch.empty_like(m_in)
    m_b = torch.empty_like(m_in) if E is not None else None
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ti = rng.integers(0, ntraj, batch)
        ki = rng.integers(0, npairs, batch)
        tit = torch.as_tensor(ti, device="cuda")
        kit = torch.as_tensor(ki, device="cuda")
        m_in.copy_(X[tit, kit])
        m_t.copy_(X[tit, kit + 1])
        if E is not None:
            m_b.copy_(E[tit, kit])
        torch.cuda.current_stream().synchronize()   # the library works on its own stream
        loss = sur.train_step(m_in, m_t, B[ti], lr=cosine_lr(s, steps, lr0), m_base=m_b)
        losses.append(loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            log(f"step {s} loss {loss:.3e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"losses": losses, "wall_s": wall, "px_per_s": steps * batch * H * W / wall}
