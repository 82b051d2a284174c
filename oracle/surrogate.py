"""FP64 reference of the convolutional surrogate: forward, backward, loss and
Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The surrogate is not
part of the paper; it is the learned multi-step proposer of this project:

    input  x (9 channels): m as a pair (hi, lo) with hi = m rounded to BF16
           (nearest, ties to even) and lo = 256 (m - hi) (m taken in FP32),
           then the applied field B / 50 mT (3)
    net    conv3x3(9->32) SiLU, 4 x [conv3x3(32->32) SiLU], conv3x3(32->3)
           ("same" size, zero padding outside the film)
    output z (3 channels), dm = scale z; proposal m' = normalize(base + dm),
           with base either m or the solver's one coarse step over the whole
           segment (computed by the caller)
    loss   mean over pixels and channels of (z - (m_target - base)/scale)^2
    Adam   lr, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected

Layout here: activations (C, H, W) per sample, weights (Cout, Cin, 3, 3),
cross-correlation: y[o, i, j] = b[o] + sum_{c,u,v} w[o, c, u, v] x[c, i+u-1, j+v-1].
"""
import numpy as np

LAYERS = ((9, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3))
B_SCALE = 0.05   # tesla: the applied field enters as B / 50 mT


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def conv3x3(x, w, b):
    """x (C, H, W), w (O, C, 3, 3), b (O,) -> (O, H, W), zero padding."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], H, W))
    for u in range(3):
        for v in range(3):
            y += np.einsum("oc,chw->ohw", w[:, :, u, v], xp[:, u:u + H, v:v + W])
    return y + b[:, None, None]


def conv3x3_backward(x, w, gy):
    """Gradients of sum(gy * conv3x3(x, w, b)) w.r.t. x, w and b."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for u in range(3):
        for v in range(3):
            gw[:, :, u, v] = np.einsum("ohw,chw->oc", gy, xp[:, u:u + H, v:v + W])
            gxp[:, u:u + H, v:v + W] += np.einsum("oc,ohw->chw", w[:, :, u, v], gy)
    return gxp[:, 1:-1, 1:-1], gw, gy.sum(axis=(1, 2))


def init_params(seed=0):
    """He-style initial weights (the last layer scaled down so the initial
    proposal is close to 'no change')."""
    rng = np.random.default_rng(seed)
    params = []
    for li, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (9 * ci))
        if li == len(LAYERS) - 1:
            std *= 0.1
        params.append((rng.standard_normal((co, ci, 3, 3)) * std, np.zeros(co)))
    return params


def round_bf16(a):
    """Nearest BF16 value of float32 a (ties to even): keep the upper 16 bits
    of the IEEE single after adding half a unit of the dropped part."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def net_input(m, B):
    """m (3, H, W), B (3,) tesla -> x (9, H, W): (hi, lo) of m, B / 50 mT."""
    H, W = m.shape[1:]
    m32 = np.asarray(m, dtype=np.float32)
    hi = round_bf16(m32)
    lo = (m32 - hi) * np.float32(256.0)
    return np.concatenate([hi.astype(np.float64), lo.astype(np.float64),
                           np.broadcast_to((np.asarray(B) / B_SCALE).reshape(3, 1, 1), (3, H, W))])


def forward(params, x):
    """Returns the output and the pre-activations of every layer."""
    acts, pre = [x], []
    h = x
    for li, (w, b) in enumerate(params):
        z = conv3x3(h, w, b)
        pre.append(z)
        h = z if li == len(params) - 1 else silu(z)
        acts.append(h)
    return h, acts, pre


def loss_and_grads(params, x, target):
    """MSE loss (mean over all outputs) and its gradients."""
    out, acts, pre = forward(params, x)
    diff = out - target
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        if li != len(params) - 1:
            g = g * silu_grad(pre[li])
        gx, gw, gb = conv3x3_backward(acts[li], params[li][0], g)
        grads[li] = (gw, gb)
        g = gx
    return loss, grads


def adam_step(params, grads, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); state holds the moment arrays."""
    new = []
    for li, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
        out = []
        for k, (p, g) in enumerate(((w, gw), (b, gb))):
            m, v = state.get((li, k), (np.zeros_like(p), np.zeros_like(p)))
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            state[(li, k)] = (m, v)
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            out.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new


def propose(params, m, B, base=None, scale=1.0):
    """m' = normalize(base + scale net(m, B)), base = m unless given."""
    z, _, _ = forward(params, net_input(m, B))
    mm = (m if base is None else base) + scale * z
    return mm / np.linalg.norm(mm, axis=0, keepdims=True)
