"""Oracle of the learned weight proposer: a 3-layer MLP (features -> 32 -> 32 -> 3, ReLU, softmax)
mapping a 5-point stencil to the three nonlinear quadrature weights, its feature map, loss and
gradients.  Plain numpy in FP64; optional emulation of BF16 rounding at the points where the GPU
kernels round (matrix-core operands).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT (only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg may use it).

Feature map (written out again, independently, in the HIP kernels), from the stencil values
s_0..s_4 (ETA5 order of ``oracle.hj``): the substencils' second differences q_r = s_r - 2 s_{r+1} +
s_{r+2} (r = 0, 1, 2) and Q = max_r |q_r|, the deviations from the centre value e_k = s_k - s_2 and
E = max_k |e_k|:
  f_0..f_2 = q_r / Q                                 (0 when Q = 0)
  f_3      = clip(log10(Q^2 / 1e-6), -8, 8) / 8      (the scale against the WENO-Z epsilon; -1 when Q = 0)
  f_4..f_7 = e_k / E for k = 0, 1, 3, 4              (0 when E = 0)
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 8, 32, 3
EPS_Z = 1e-6


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest even on the top 16 bits of the float32), back to float64."""
    x = np.asarray(a, dtype=np.float32).copy()
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def features(S: np.ndarray) -> np.ndarray:
    S = np.asarray(S, dtype=float)
    q = np.stack([S[..., r] - 2.0 * S[..., r + 1] + S[..., r + 2] for r in range(3)], axis=-1)
    Q = np.abs(q).max(axis=-1, keepdims=True)
    e = S - S[..., 2:3]
    E = np.abs(e).max(axis=-1, keepdims=True)
    f = np.zeros(S.shape[:-1] + (NIN,))
    f[..., 0:3] = np.where(Q > 0, q / np.where(Q > 0, Q, 1.0), 0.0)
    with np.errstate(divide="ignore"):
        lg = np.log10(np.where(Q[..., 0] > 0, Q[..., 0] ** 2 / EPS_Z, 1e-300))
    f[..., 3] = np.clip(lg, -8.0, 8.0) / 8.0
    f[..., 4:8] = np.where(E > 0, e[..., [0, 1, 3, 4]] / np.where(E > 0, E, 1.0), 0.0)
    return f


def init_params(seed: int = 0):
    """He-initialised weights (W: (out, in)), zero biases."""
    g = np.random.default_rng(seed)
    W1 = g.standard_normal((NH, NIN)) * np.sqrt(2.0 / NIN)
    W2 = g.standard_normal((NH, NH)) * np.sqrt(2.0 / NH)
    W3 = g.standard_normal((NOUT, NH)) * np.sqrt(1.0 / NH)
    return dict(W1=W1, b1=np.zeros(NH), W2=W2, b2=np.zeros(NH), W3=W3, b3=np.zeros(NOUT))


def forward(p, X, emulate_bf16: bool = False):
    """Returns (omega, cache).  With emulate_bf16, the operands of every matrix product (inputs,
    weights, hidden activations) are rounded to BF16 first; sums stay exact (FP64)."""
    r = bf16 if emulate_bf16 else (lambda a: a)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    x0 = r(X)
    z1 = x0 @ W1.T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1r = r(h1)
    z2 = h1r @ W2.T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    h2r = r(h2)
    z3 = h2r @ W3.T + p["b3"]
    z3 = z3 - z3.max(axis=-1, keepdims=True)
    e = np.exp(z3)
    om = e / e.sum(axis=-1, keepdims=True)
    return om, dict(x0=x0, z1=z1, h1r=h1r, z2=z2, h2r=h2r, om=om, W2=W2, W3=W3)


def loss(om, target) -> float:
    """Mean over the batch of the squared error of the three weights."""
    return float(((om - target) ** 2).sum(axis=-1).mean())


def backward(p, cache, target, emulate_bf16: bool = False, with_upstream: bool = False):
    """Gradients of ``loss`` w.r.t. every parameter (chain rule written out layer by layer).  With
    emulate_bf16 the upstream gradients entering matrix products are BF16-rounded too.  With
    with_upstream, also returns the gradients w.r.t. the pre-activations (z3, z2, z1) as they enter
    the products (for error bounds in tests)."""
    r = bf16 if emulate_bf16 else (lambda a: a)
    n = target.shape[0]
    om = cache["om"]
    g_om = 2.0 * (om - target) / n
    # softmax Jacobian: dz_k = om_k (g_k - sum_j g_j om_j)
    g_z3 = om * (g_om - (g_om * om).sum(axis=-1, keepdims=True))
    g3r = r(g_z3)
    gW3 = g3r.T @ cache["h2r"]
    gb3 = g_z3.sum(axis=0)
    g_h2 = g3r @ cache["W3"]
    g_z2 = g_h2 * (cache["z2"] > 0)
    g2r = r(g_z2)
    gW2 = g2r.T @ cache["h1r"]
    gb2 = g_z2.sum(axis=0)
    g_h1 = g2r @ cache["W2"]
    g_z1 = g_h1 * (cache["z1"] > 0)
    g1r = r(g_z1)
    gW1 = g1r.T @ cache["x0"]
    gb1 = g_z1.sum(axis=0)
    grads = dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3)
    if with_upstream:
        return grads, dict(z3=g3r, z2=g2r, z1=g1r)
    return grads


def adam_step(p, g, state, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba) of every parameter, in place; state holds m, v and the step."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
