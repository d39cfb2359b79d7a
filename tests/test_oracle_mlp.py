"""Pins of the FP64 surrogate oracle: its hand-written backward pass against
central finite differences, and one Adam step against the update formula of
Kingma & Ba evaluated element by element."""
import numpy as np

from oracle import mlp as M


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = M.init_params(11)
    xh = rng.uniform(-1, 1, size=(16, 4))
    th = rng.normal(size=(16, 8))
    loss, g = M.loss_and_grad(p, xh, th)
    idx = np.concatenate([rng.choice(M.N_TRAINABLE, 60, replace=False), [M.N_TRAINABLE - 1, 0, 256, 9152]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss_and_grad(pp, xh, th)[0] - M.loss_and_grad(pm, xh, th)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])
    assert np.all(g[M.N_TRAINABLE:] == 0)


def test_adam_step_formula():
    rng = np.random.default_rng(4)
    p = rng.normal(size=M.N_PARAMS)
    g = rng.normal(size=M.N_PARAMS)
    m = rng.normal(size=M.N_PARAMS) * 0.1
    v = np.abs(rng.normal(size=M.N_PARAMS)) * 0.1
    p2, m2, v2 = M.adam_step(p, g, m, v, t=3, lr=1e-2)
    for i in [0, 100, 9159]:
        mi = 0.9 * m[i] + 0.1 * g[i]
        vi = 0.999 * v[i] + 0.001 * g[i] ** 2
        step = 1e-2 * (mi / (1 - 0.9 ** 3)) / (np.sqrt(vi / (1 - 0.999 ** 3)) + 1e-8)
        assert abs(p2[i] - (p[i] - step)) < 1e-14
    assert np.array_equal(p2[M.N_TRAINABLE:], p[M.N_TRAINABLE:])


def test_prediction_denormalises():
    p = M.init_params(2, mu=np.arange(8.0), sigma=np.full(8, 2.0))
    x = np.array([[1.0, 0.3, 0.2, 0.65]])  # already canonical (u_x >= u_y >= 0)
    y, _ = M.forward(p, M.normalize_inputs(x))
    assert np.allclose(M.predict(p, x), np.arange(8.0) + 2.0 * y)
    # a reflected state: sign flips of the odd multipliers, nothing else
    xr = np.array([[1.0, -0.3, 0.2, 0.65]])
    flip = np.array([1, -1, 1, 1, -1, 1, -1, 1])
    assert np.allclose(M.predict(p, xr), flip * (np.arange(8.0) + 2.0 * y))


def test_canonical_map_is_the_lattice_symmetry():
    """the reflection/swap map of the multipliers agrees with the oracle's
    Newton solution at the mapped states (exact symmetry of Eq. exponential
    on the D2Q21 lattice)"""
    from oracle.oracle import Oracle
    o = Oracle("D2Q21", "DDF_NEWTON", T0=0.65, gamma=1.4)
    states = np.array([[1.0, -0.4, 0.7, 0.6], [1.0, 0.9, -0.3, 0.8], [1.0, -0.5, -0.6, 0.7]])
    lam = np.array([o.newton(s[1:3], s[3])[1] for s in states])
    xc, lc, unflip = M.canonicalize(states, lam)
    assert np.all(xc[:, 1] >= xc[:, 2]) and np.all(xc[:, 2] >= 0)
    for k in range(len(states)):
        _, lref = o.newton(xc[k, 1:3], xc[k, 3])
        assert np.max(np.abs(lc[k] - lref)) < 1e-9
    assert np.max(np.abs(unflip(lc) - lam)) < 1e-15
