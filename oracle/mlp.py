"""FP64 CPU reference of the multiplier surrogate (TEST INFRASTRUCTURE ONLY).

The surrogate maps the macroscopic state (rho, u_x, u_y, T) of a D2Q21 cell to
the eight Lagrange multipliers of the numerical equilibrium (App. A.2, Eq.
exponential and the eight constraints G(0)..G(3)).  Network: 4 -> 64 -> 64
-> 64 -> 8, SiLU on the hidden layers, linear output, on normalised inputs
and outputs; loss = mean Huber loss (delta 0.5) over samples and outputs of
the normalised outputs (the multipliers are heavy-tailed near the boundary of
the realisable moments, so a quadratic loss lets a few states dominate); Adam.

Parameters are one packed FP32/FP64 vector (the same packing the HIP library
uses for its master weights):
  W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[8][64] b4[8]
  mu[8] sigma[8]        (output de-normalisation: lambda = mu + sigma * y)
Input normalisation: ((rho - 2.6) / 2.4, u_x / 2.5, u_y / 2.5, (T - 1.75) / 1.25).
"""
from __future__ import annotations

import numpy as np

SIZES = [("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 64)),
         ("b3", (64,)), ("W4", (8, 64)), ("b4", (8,)), ("mu", (8,)), ("sigma", (8,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 9176
N_TRAINABLE = N_PARAMS - 16


def unpack(p):
    out, k = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[k:k + n].reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def normalize_inputs(x):
    x = np.asarray(x, dtype=np.float64)
    return np.stack([(x[:, 0] - 2.6) / 2.4, x[:, 1] / 2.5, x[:, 2] / 2.5, (x[:, 3] - 1.75) / 1.25], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, xh):
    """normalised inputs [n, 4] -> normalised outputs [n, 8] and the cache."""
    P = unpack(p)
    z1 = xh @ P["W1"].T + P["b1"]
    h1 = silu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = silu(z2)
    z3 = h2 @ P["W3"].T + P["b3"]
    h3 = silu(z3)
    y = h3 @ P["W4"].T + P["b4"]
    return y, (xh, z1, h1, z2, h2, z3, h3)


def canonicalize(x, lam=None):
    """map states to the octant u_x >= u_y >= 0 by the reflections of the
    lattice; the multipliers transform with them (x <-> y exchange of the
    components, sign of the components odd in x or y).  Returns the mapped
    states, mapped multipliers (if given) and the inverse map."""
    x = np.array(x, dtype=np.float64)
    sx, sy = x[:, 1] < 0, x[:, 2] < 0
    x[:, 1], x[:, 2] = np.abs(x[:, 1]), np.abs(x[:, 2])
    sw = x[:, 2] > x[:, 1]
    x[sw, 1], x[sw, 2] = x[sw, 2].copy(), x[sw, 1].copy()

    def flip(l):
        l = np.array(l, dtype=np.float64)
        for m, idx in [(sx, [1, 4, 6]), (sy, [2, 4, 7])]:
            for k in idx:
                l[m, k] = -l[m, k]
        for a, b in [(1, 2), (3, 5), (6, 7)]:
            l[sw, a], l[sw, b] = l[sw, b].copy(), l[sw, a].copy()
        return l

    def unflip(l):
        l = np.array(l, dtype=np.float64)
        for a, b in [(1, 2), (3, 5), (6, 7)]:
            l[sw, a], l[sw, b] = l[sw, b].copy(), l[sw, a].copy()
        for m, idx in [(sx, [1, 4, 6]), (sy, [2, 4, 7])]:
            for k in idx:
                l[m, k] = -l[m, k]
        return l

    return x, (None if lam is None else flip(lam)), unflip


def predict(p, x):
    """multipliers from macroscopic states [n, 4] (rho, u_x, u_y, T): the
    network is evaluated on the canonical state and mapped back."""
    P = unpack(p)
    xc, _, unflip = canonicalize(x)
    y, _ = forward(p, normalize_inputs(xc))
    return unflip(P["mu"] + P["sigma"] * y)


HUBER = 0.5


def loss_and_grad(p, xh, th):
    """mean over samples and outputs of the Huber loss of y - t, and its
    gradient with the same packing (zero for mu and sigma)."""
    P = unpack(p)
    y, (xh, z1, h1, z2, h2, z3, h3) = forward(p, xh)
    n = xh.shape[0]
    r = y - th
    a = np.abs(r)
    loss = float(np.mean(np.where(a <= HUBER, 0.5 * r * r, HUBER * (a - 0.5 * HUBER))))
    d4 = np.clip(r, -HUBER, HUBER) / (n * 8)
    g = {"W4": d4.T @ h3, "b4": d4.sum(0)}
    d3 = (d4 @ P["W4"]) * dsilu(z3)
    g["W3"], g["b3"] = d3.T @ h2, d3.sum(0)
    d2 = (d3 @ P["W3"]) * dsilu(z2)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ P["W2"]) * dsilu(z1)
    g["W1"], g["b1"] = d1.T @ xh, d1.sum(0)
    g["mu"] = np.zeros(8)
    g["sigma"] = np.zeros(8)
    return loss, pack(g)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """one Adam update (Kingma & Ba 2015) of the trainable entries; t counts
    from 1; returns new (p, m, v)."""
    p, m, v = p.copy(), m.copy(), v.copy()
    k = N_TRAINABLE
    m[:k] = beta1 * m[:k] + (1 - beta1) * g[:k]
    v[:k] = beta2 * v[:k] + (1 - beta2) * g[:k] * g[:k]
    mh = m[:k] / (1 - beta1 ** t)
    vh = v[:k] / (1 - beta2 ** t)
    p[:k] -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def init_params(seed, mu=None, sigma=None):
    """He-style uniform initialisation (the HIP library takes weights set by
    the caller, so both sides can start from the same vector)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            fan_in = shape[1]
            lim = np.sqrt(6.0 / fan_in) * 0.5
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    d["mu"] = np.zeros(8) if mu is None else mu
    d["sigma"] = np.ones(8) if sigma is None else sigma
    return pack(d)
