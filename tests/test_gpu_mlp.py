"""GPU tests of the multiplier surrogate: Newton labels against the oracle's
Newton, BF16-MFMA forward and gradients against the FP64 CPU MLP, training,
the surrogate-corrected collide kernel against the FP64 oracle, and what the
trained network gains over the cold-started Newton solve."""
import time

import numpy as np
import pytest

from gpu_util import compare, run_pair, say
from oracle import mlp as M
from oracle.oracle import Oracle
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu


def d2q21_ctx(**kw):
    w = W.airfoil(scale=32, steps=1)
    return B.LBM.from_workload(w, storage="fp32", **kw)


def realizable(o, u, T):
    """a positive discrete distribution with the eight target moments exists
    (linear feasibility with f_i >= 1e-9)"""
    from scipy.optimize import linprog
    c = o.c[:, :2].astype(float)
    x, y = c[:, 0], c[:, 1]
    n2 = x * x + y * y
    A = np.stack([np.ones(o.Q), x, y, x * x, x * y, y * y, x * n2, y * n2])
    uu = u[0] ** 2 + u[1] ** 2
    M = np.array([1, u[0], u[1], u[0] ** 2 + T, u[0] * u[1], u[1] ** 2 + T, u[0] * (uu + 4 * T), u[1] * (uu + 4 * T)])
    r = linprog(np.zeros(o.Q), A_eq=A, b_eq=M, bounds=[(1e-9, None)] * o.Q, method="highs")
    return r.status == 0


def test_labels_match_oracle_newton():
    """GPU Newton labels: accepted exactly where the moments are realisable,
    and equal to the oracle's multipliers where both converge."""
    s = d2q21_ctx(newton_max_it=60)
    x = W.mlp_samples(512, seed=21)
    lam, ok, it = s.mlp_label(x)
    o = Oracle("D2Q21", "DDF_NEWTON", T0=0.65, gamma=1.4)
    agree_lp, both, maxdiff = 0, 0, 0.0
    for k in range(len(x)):
        if realizable(o, x[k, 1:3], x[k, 3]) == bool(ok[k]):
            agree_lp += 1
        ito, lo = o.newton(x[k, 1:3], x[k, 3], max_it=60)
        if ito >= 0 and ok[k]:
            both += 1
            maxdiff = max(maxdiff, float(np.max(np.abs(lo - lam[k]))))
    say(f"[mlp] labels: accepted {ok.mean():.3f}, agreement with realisability {agree_lp / len(x):.4f}, "
        f"{both} converged on both sides, max |dlambda| {maxdiff:.2e}")
    assert agree_lp >= 0.97 * len(x)
    assert both >= 0.95 * ok.sum()
    assert maxdiff < 1e-8
    assert 0.15 < ok.mean() < 0.6


def test_forward_and_gradient_against_fp64_oracle():
    rng = np.random.default_rng(8)
    p = M.init_params(13, mu=rng.normal(size=8), sigma=np.abs(rng.normal(size=8)) + 0.5)
    s = d2q21_ctx()
    s.mlp_set_weights(p.astype(np.float32))
    x = W.mlp_samples(256, seed=3)
    ref = M.predict(p, x)
    got = s.mlp_predict(x)
    sig = p[M.N_PARAMS - 8:]
    err = np.max(np.abs((got - ref) / sig))
    say(f"[mlp] forward: max normalised error {err:.2e}")
    assert err < 3e-2
    xh = M.normalize_inputs(x)
    th = rng.normal(size=(256, 8))
    loss_ref, g_ref = M.loss_and_grad(p, xh, th)
    loss, g = s.mlp_grad(xh, th)
    g_ref = g_ref[: M.N_TRAINABLE]
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    cos = float(np.dot(g, g_ref) / (np.linalg.norm(g) * np.linalg.norm(g_ref)))
    say(f"[mlp] gradient: loss {loss:.6f} vs {loss_ref:.6f}, rel L2 {rel:.3e}, cosine {cos:.6f}")
    assert np.count_nonzero(np.abs(th) > 3) > 0  # both branches of the Huber loss are exercised
    assert abs(loss - loss_ref) < 2e-2 * loss_ref
    assert rel < 5e-2 and cos > 0.998
    # per-layer check, so that a transposed or misplaced block fails
    offs = [(0, 256), (256, 320), (320, 4416), (4416, 4480), (4480, 8576), (8576, 8640), (8640, 9152), (9152, 9160)]
    for a, b in offs:
        r = np.linalg.norm(g[a:b] - g_ref[a:b]) / max(np.linalg.norm(g_ref[a:b]), 1e-30)
        assert r < 8e-2, (a, b, r)


@pytest.fixture(scope="module")
def trained():
    s = d2q21_ctx(newton_max_it=60)
    x = W.mlp_samples(400_000, seed=5)
    t0 = time.perf_counter()
    lam, ok, it = s.mlp_label(x)
    t1 = time.perf_counter()
    hist = s.mlp_train(x[ok], lam[ok], epochs=30, batch=1024, lr=1e-2, seed=5)
    t2 = time.perf_counter()
    say(f"[mlp] labelled {len(x)} states in {t1 - t0:.2f} s ({ok.sum()} accepted), trained 30 epochs in "
        f"{t2 - t1:.2f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    return s.mlp_get_weights(), hist, x[ok][:4096], lam[ok][:4096]


def test_training_reduces_loss(trained):
    """the Huber loss falls and the typical error of the trained network is a
    few percent of the spread of each multiplier (the heavy tail near the
    boundary of realisable moments stays large; Newton corrects it)"""
    w, hist, xs, ls = trained
    assert hist[-1] < 0.5 * hist[0]
    p = w.astype(np.float64)
    pred = M.predict(p, xs)
    sig = p[M.N_PARAMS - 8:]
    r = np.abs((pred - ls) / sig)
    say(f"[mlp] trained network on training states: normalised median |err| {np.median(r):.3e}, "
        f"p90 {np.percentile(r, 90):.3e}")
    assert np.median(r) < 0.05


@pytest.mark.parametrize("variant", ["DDF_MLP_NEWTON"])
def test_surrogate_collision_parity(trained, variant):
    """one Newton correction + fallback stays within relative L2 1e-5 of the
    Newton path at the same (FP32) storage -- the bar on the surrogate --
    and so within that of the Newton path's own FP64-oracle agreement"""
    w = W.airfoil(scale=16, steps=20)
    wts = trained[0]
    probe = B.LBM.from_workload(w, storage="fp32", host_only=True)
    coords, level = probe.coords_levels()
    m0 = w.initial_moments(coords, level)
    o2 = Oracle.from_workload(w)
    o2.init(m0)
    s2 = B.LBM.from_workload(w, storage="fp32")
    s2.init(m0)
    s3 = B.LBM(w.lattice, variant, "fp32", nu_finest=w.nu_finest, T0=w.T0, gamma=w.gamma, sensor_A=w.sensor_A,
               sensor_on=w.sensor_on, newton_tol=w.newton_tol, newton_max_it=w.newton_max_it)
    s3.grid(w.dim, w.ext, w.n_levels, w.refine, w.solid, w.faces)
    s3.mlp_set_weights(wts)
    s3.init(m0)
    for k in range(20):
        for face, f in w.schedule(k).items():
            o2.set_face(face, f)
            s2.set_face(face, f)
            s3.set_face(face, f)
        o2.step(1)
        s2.step(1)
        s3.step(1)
    mo = o2.moments()
    e_newton = compare(s2.moments(), mo, level, 2)
    e_mlp = compare(s3.moments(), mo, level, 2)
    e_vs = compare(s3.moments(), s2.moments(), level, 2)
    st = s3.stats()
    say(f"[mlp] airfoil/16 20 steps: Newton FP32 {e_newton}; surrogate+Newton FP32 {e_mlp}; "
        f"surrogate vs Newton {e_vs}; fallbacks {st['mlp_fallbacks']} of {sum(st['updates'])} updates")
    for k in ("rho", "u", "T"):
        # the bar: relative L2 <= 1e-5 against Newton at the same storage
        assert e_vs[k] < 1e-5, (k, e_vs[k])
        # against the FP64 oracle the two paths then differ by at most that
        assert e_mlp[k] <= e_newton[k] + 1e-5, (k, e_mlp[k], e_newton[k])
    assert st["newton_failures"] == 0


def test_surrogate_iterations_between_cold_and_warm_newton(trained):
    """Where the network's multipliers stand as a first Newton iterate: far
    better than the cold start (lambda = 0 every step), worse than the
    method's own warm start (the previous step's multipliers), which is why
    variant (c) is slower than warm-started Newton on the developed flow.
    Iterations are asserted both ways on the same states; collide times are
    reported, not asserted (on this small grid launches and latency
    dominate; bench.py times the full-size airfoil)."""
    wts = trained[0]
    w = W.airfoil(scale=8, steps=10)

    def run(coll, warm):
        s = B.LBM(w.lattice, coll, "fp32", nu_finest=w.nu_finest, T0=w.T0, gamma=w.gamma, sensor_A=w.sensor_A,
                  sensor_on=w.sensor_on, newton_tol=w.newton_tol, newton_max_it=w.newton_max_it, warm_start=warm)
        s.grid(w.dim, w.ext, w.n_levels, w.refine, w.solid, w.faces)
        if coll != "DDF_NEWTON":
            s.mlp_set_weights(wts)
        s.init_workload(w)
        s.step(2)
        s.sync()
        s.profile(True)
        s.step(8)
        s.sync()
        ms = sum(s.profile_read(l)[1] for l in range(w.n_levels))
        st = s.stats()
        return ms, st

    t_cold, st_cold = run("DDF_NEWTON", False)
    t_warm, st_warm = run("DDF_NEWTON", True)
    t_mlp, st_mlp = run("DDF_MLP_NEWTON", True)
    say(f"[mlp] collide time over 8 coarse steps: cold Newton {t_cold:.2f} ms ({st_cold['newton_iterations']} it), "
        f"warm Newton {t_warm:.2f} ms ({st_warm['newton_iterations']} it), surrogate+Newton {t_mlp:.2f} ms "
        f"({st_mlp['newton_iterations']} it incl. the corrections, {st_mlp['mlp_fallbacks']} fallbacks); "
        f"speed-up vs cold {t_cold / t_mlp:.2f}x, vs warm {t_warm / t_mlp:.2f}x")
    assert st_mlp["newton_iterations"] < 0.5 * st_cold["newton_iterations"]
    assert st_mlp["newton_iterations"] > st_warm["newton_iterations"]
    assert st_mlp["newton_failures"] == 0 and st_cold["newton_failures"] == 0


def test_surrogate_alone_misses_the_constraints(trained):
    """Variant (b), the network's multipliers used as they are: the
    equilibrium it builds does not meet the moment constraints, so mass,
    momentum and energy are not conserved by the collision and the run
    drifts from the oracle.  Reported per coarse step on the scaled airfoil
    (a closed box would be cleaner, but the airfoil is the workload): the
    relative L2 against the oracle, the constraint residual of the network's
    multipliers at the same states (max |G_a| / rho after one evaluation,
    the fallback test of variant (c)), and the share of colliding states
    outside the training box.  The bar of 1e-5 is out of reach for (b): on
    this grid the run also leaves the representable states within a few
    steps and latches a numeric failure (non-finite cells), as the
    full-size airfoil does; the diagnosis uses the last finite state."""
    w = W.airfoil(scale=16, steps=12)
    wts = trained[0]
    o = Oracle.from_workload(w)
    s = B.LBM(w.lattice, "DDF_MLP", "fp32", nu_finest=w.nu_finest, T0=w.T0, gamma=w.gamma, sensor_A=w.sensor_A,
              sensor_on=w.sensor_on, newton_tol=w.newton_tol, newton_max_it=w.newton_max_it)
    s.grid(w.dim, w.ext, w.n_levels, w.refine, w.solid, w.faces)
    s.mlp_set_weights(wts)
    coords, level = s.coords_levels()
    m0 = w.initial_moments(coords, level)
    o.init(m0)
    s.init(m0)
    errs = []
    m = s.moments()
    failed_at = None
    for k in range(12):
        for face, f in w.schedule(k).items():
            o.set_face(face, f)
            s.set_face(face, f)
        o.step(1)
        s.step(1)
        try:
            mk = s.moments()
        except B.LbmError as e:
            assert e.code == -6  # the numeric latch, not another failure
            failed_at = k
            break
        m = mk
        errs.append(compare(m, o.moments(), level, 2)["rho"])
    ok = np.isfinite(m[0])
    x = np.stack([m[0][ok], m[1][ok], m[2][ok], m[3][ok]], axis=1)
    speed = np.hypot(x[:, 1], x[:, 2])
    outside = float(np.mean((x[:, 0] < 0.2) | (x[:, 0] > 5.0) | (speed > 2.5) | (x[:, 3] < 0.5) | (x[:, 3] > 3.0)))
    # residual of the network's multipliers at the library's states
    lam = s.mlp_predict(x)
    xi = o.c[:, :2].astype(np.float64)
    mv = np.stack([np.ones(len(xi)), xi[:, 0], xi[:, 1], xi[:, 0] ** 2, xi[:, 0] * xi[:, 1], xi[:, 1] ** 2,
                   xi[:, 0] * (xi ** 2).sum(1), xi[:, 1] * (xi ** 2).sum(1)], axis=1)

    def residual(st, lm):
        # max_a |G_a| / rho of the exponential equilibrium (Eq. exponential)
        ux, uy, T = st[1], st[2], st[3]
        u2 = ux * ux + uy * uy
        tgt = np.array([1.0, ux, uy, ux * ux + T, ux * uy, uy * uy + T, ux * (u2 + 4 * T), uy * (u2 + 4 * T)])
        e = np.exp(-(1.0 + mv @ lm))
        return float(np.max(np.abs(e @ mv - tgt)))

    with np.errstate(over="ignore", invalid="ignore"):
        res = np.array([residual(x[i], lam[i]) for i in range(0, len(x), max(1, len(x) // 400))])
        # the same at the initial (developing, realisable) states
        x0 = np.stack([m0[0], m0[1], m0[2], m0[3]], axis=1)
        lam0 = s.mlp_predict(x0)
        res0 = np.array([residual(x0[i], lam0[i]) for i in range(0, len(x0), max(1, len(x0) // 400))])
    say(f"[mlp] variant (b) on airfoil/16: rel L2(rho) by coarse step {np.array(errs)}; non-finite cells latched "
        f"at coarse step {failed_at}; at the last finite state: share of states outside the training box "
        f"{outside:.3e}, network constraint residual median {np.nanmedian(res):.2e}, non-finite "
        f"{np.mean(~np.isfinite(res)):.3f}; at the initial states median {np.median(res0):.2e}, "
        f"max {np.max(res0):.2e}")
    # (b) alone does not meet the bar: it diverges, or drifts beyond 1e-5
    assert failed_at is not None or errs[-1] > 1e-5
    # its multipliers violate the constraints (the fallback threshold of (c)
    # is 1e-10), already at the initial states
    assert np.median(res0) > 1e-10
    s.close()
