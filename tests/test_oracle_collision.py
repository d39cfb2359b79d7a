"""Pins of the oracle's equilibria and collisions (App. A.2 / A.3) against
closed forms, moment identities, the paper's printed fourth-order
non-equilibrium recursion, the DDF closure, the kinetic sensor table and the
Newton constraint residual."""
import itertools
import math

import numpy as np
import pytest

from oracle.oracle import Oracle

rng = np.random.default_rng(1234)


def moms(o, f, degree):
    """raw moments sum_i f_i xi^p for all multi-indices p with |p| <= degree"""
    xi = o.c[:, : o.D].astype(np.float64)
    out = {}
    for p in itertools.product(range(degree + 1), repeat=o.D):
        if sum(p) <= degree:
            out[p] = float((f * np.prod([xi[:, d] ** p[d] for d in range(o.D)], axis=0)).sum())
    return out


def gauss_raw(n, mu, var):
    """E[X^n], X ~ N(mu, var), by expanding (mu + sqrt(var) Z)^n."""
    from math import comb
    tot = 0.0
    for k in range(0, n + 1, 2):
        dfact = 1.0
        for j in range(1, k, 2):
            dfact *= j
        tot += comb(n, k) * mu ** (n - k) * var ** (k // 2) * dfact
    return tot


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_isothermal_equilibrium_is_product_form(name):
    """With the Hermite set {0,1,2}^D the equilibrium factorises into the D1Q3
    second-order equilibria (textbook product form)."""
    o = Oracle(name, "BGK", nu_finest=0.1)
    for _ in range(5):
        rho = 0.8 + 0.4 * rng.random()
        u = 0.2 * (rng.random(o.D) - 0.5)
        fe, _, _ = o.feq(rho, u)
        cs2 = 1.0 / 3.0
        ref = np.array([o.w[i] * rho * np.prod([1 + o.c[i, d] * u[d] / cs2
                                                 + (o.c[i, d] ** 2 - cs2) * u[d] ** 2 / (2 * cs2 ** 2)
                                                 for d in range(o.D)]) for i in range(o.Q)])
        assert np.max(np.abs(fe - ref)) < 1e-15
        m = moms(o, fe, 2)
        assert abs(m[(0,) * o.D] - rho) < 1e-14
        for d in range(o.D):
            e = [0] * o.D
            e[d] = 1
            assert abs(m[tuple(e)] - rho * u[d]) < 1e-15
        for a in range(o.D):
            for b in range(o.D):
                e = [0] * o.D
                e[a] += 1
                e[b] += 1
                ref2 = rho * (u[a] * u[b] + (cs2 if a == b else 0.0))
                assert abs(m[tuple(e)] - ref2) < 1e-14


def test_d2q37_thermal_equilibrium_gaussian_moments():
    """D2Q37 integrates degree-9 monomials exactly, so every moment of order
    <= 4 of the fourth-order thermal equilibrium equals the Maxwellian's."""
    o = Oracle("D2Q37", "DDF_POLY", T0=1.0, gamma=1.4)
    for _ in range(6):
        rho = 0.2 + rng.random()
        u = 0.6 * (rng.random(2) - 0.5)
        T = 0.6 + 0.6 * rng.random()
        fe, ge, _ = o.feq(rho, u, T)
        m = moms(o, fe, 4)
        for p, v in m.items():
            ref = rho * gauss_raw(p[0], u[0], T) * gauss_raw(p[1], u[1], T)
            assert abs(v - ref) < 3e-14 * max(1.0, abs(ref)), (p, v, ref)
        # DDF closure, Eqs. gEq and polyTemp: g_eq = (2 Cv - D) T f_eq and the
        # temperature recomputed from (f_eq, g_eq) is T
        Cv = 1.0 / (1.4 - 1.0)
        assert np.max(np.abs(ge - (2 * Cv - 2) * T * fe)) < 1e-15
        xi2 = (o.c[:, :2].astype(float) ** 2).sum(1)
        Trec = ((xi2 * fe + ge).sum() - rho * (u ** 2).sum()) / (2 * rho * Cv)
        assert abs(Trec - T) < 1e-13


def hermite_project(o, f, m):
    """a_m = sum_i H_m(xi_i) f_i with H from D1Q3 factors (orthogonal basis of
    the product lattices)."""
    cs2 = o.cs2
    h = {0: lambda x: 1.0 + 0 * x, 1: lambda x: x, 2: lambda x: x * x - cs2}
    H = np.ones(o.Q)
    for d in range(o.D):
        H = H * h[m[d]](o.c[:, d].astype(float))
    return float((H * f).sum())


def rr_case(o, tau):
    rho = 0.9 + 0.2 * rng.random()
    u = 0.15 * (rng.random(o.D) - 0.5)
    fe, _, _ = o.feq(rho, u)
    f = fe * (1.0 + 0.05 * (rng.random(o.Q) - 0.5))
    fs, _, _, _ = o.collide(tau, f)
    return f, fs


def test_rr_matches_printed_fourth_order_forms_d2q9():
    """The paper prints the N=4 non-equilibrium moments explicitly (after its
    Malaspinas recursion); the oracle's post-collision moments must carry
    exactly those a_neq."""
    o = Oracle("D2Q9", "RR", nu_finest=0.1)
    tau = 0.8
    for _ in range(5):
        f, fs = rr_case(o, tau)
        rho = f.sum()
        ux, uy = (f * o.c[:, 0]).sum() / rho, (f * o.c[:, 1]).sum() / rho
        fe, _, _ = o.feq(rho, (ux, uy))
        # a^(2)_neq from the populations
        axx = hermite_project(o, f - fe, (2, 0))
        axy = hermite_project(o, f - fe, (1, 1))
        ayy = hermite_project(o, f - fe, (0, 2))
        # printed forms (App. A.2): third and fourth order
        a_xxy = 2 * ux * axy + uy * axx
        a_yyx = 2 * uy * axy + ux * ayy
        a_xxyy = 2 * (ux * a_yyx + uy * a_xxy) - ux ** 2 * ayy - uy ** 2 * axx - 4 * ux * uy * axy
        k = 1.0 - 1.0 / tau
        for m, an in [((2, 0), axx), ((1, 1), axy), ((0, 2), ayy), ((2, 1), a_xxy),
                      ((1, 2), a_yyx), ((2, 2), a_xxyy)]:
            aeq = rho * ux ** m[0] * uy ** m[1]
            got = hermite_project(o, fs, m)
            assert abs(got - (aeq + k * an)) < 1e-15, m


def test_rr_d3q27_pair_sum_closed_form():
    """For D3Q27 every kept a_neq equals the closed pair sum
    sum_{p<q} a2_{ap aq} prod_{k != p,q} u_ak, which solves the recursion."""
    o = Oracle("D3Q27", "RR", nu_finest=0.1)
    tau = 0.7
    for _ in range(3):
        f, fs = rr_case(o, tau)
        rho = f.sum()
        u = np.array([(f * o.c[:, d]).sum() / rho for d in range(3)])
        fe, _, _ = o.feq(rho, u)
        a2 = np.zeros((3, 3))
        for a in range(3):
            for b in range(3):
                m = [0, 0, 0]
                m[a] += 1
                m[b] += 1
                a2[a, b] = hermite_project(o, f - fe, m)
        for m in itertools.product(range(3), repeat=3):
            tup = [d for d in range(3) for _ in range(m[d])]
            n = len(tup)
            an = 0.0
            for p, q in itertools.combinations(range(n), 2):
                pu = 1.0
                for k in range(n):
                    if k not in (p, q):
                        pu *= u[tup[k]]
                an += a2[tup[p], tup[q]] * pu
            aeq = rho * np.prod(u ** np.array(m))
            got = hermite_project(o, fs, m)
            assert abs(got - (aeq + (1 - 1 / tau) * an)) < 2e-15, m


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27", "D2Q13", "D2Q21"])
@pytest.mark.parametrize("coll", ["BGK", "RR"])
def test_collision_conserves_and_fixes_equilibrium(name, coll):
    o = Oracle(name, coll, nu_finest=0.1)
    f, fs = rr_case(o, 0.73)
    xi = o.c[:, : o.D].astype(float)
    assert abs(fs.sum() - f.sum()) < 1e-14
    assert np.max(np.abs(xi.T @ fs - xi.T @ f)) < 1e-15
    rho = f.sum()
    u = xi.T @ f / rho
    fe, _, _ = o.feq(rho, u)
    fs2, _, _, _ = o.collide(0.73, fe)
    assert np.max(np.abs(fs2 - fe)) < 1e-15
    fs1, _, _, _ = o.collide(1.0, f)  # tau = 1: full relaxation
    assert np.max(np.abs(fs1 - fe)) < 1e-15


@pytest.mark.parametrize("name", ["D2Q13", "D2Q21"])
def test_rr_third_order_lattices_by_least_squares(name):
    """D2Q13 and D2Q21 expand to full third order and no further (Table
    lattices_hermite, App. A.2).  The Hermite coefficients of a
    post-collision state are recovered by least squares on the basis
    w_i H_m(xi_i), |m| <= 3 (13 or 21 equations, 10 unknowns): the state must
    lie in that span, and the coefficients must be the equilibrium moments
    rho u^m plus (1 - 1/tau) times the printed non-equilibrium forms, with
    a^(2)_neq taken from the raw second moment of the populations (a route
    the oracle does not take: it projects f - f_eq)."""
    o = Oracle(name, "RR", nu_finest=0.1)
    cs2 = o.cs2
    h = [lambda x: 1.0 + 0 * x, lambda x: x, lambda x: x * x - cs2, lambda x: (x * x - 3 * cs2) * x]
    xi = o.c[:, :2].astype(float)
    ms = [(mx, n - mx) for n in range(4) for mx in range(n, -1, -1)]
    A = np.stack([o.w * h[mx](xi[:, 0]) * h[my](xi[:, 1]) for mx, my in ms], axis=1)
    assert np.linalg.matrix_rank(A) == len(ms)
    tau = 0.77
    k = 1.0 - 1.0 / tau
    for _ in range(4):
        f, fs = rr_case(o, tau)
        rho = f.sum()
        ux, uy = xi.T @ f / rho
        P = np.einsum("i,ia,ib->ab", f, xi, xi)
        axx = P[0, 0] - rho * ux * ux - rho * cs2
        axy = P[0, 1] - rho * ux * uy
        ayy = P[1, 1] - rho * uy * uy - rho * cs2
        an = {(2, 0): axx, (1, 1): axy, (0, 2): ayy,
              (3, 0): 3 * ux * axx, (2, 1): 2 * ux * axy + uy * axx,
              (1, 2): 2 * uy * axy + ux * ayy, (0, 3): 3 * uy * ayy}
        b, *_ = np.linalg.lstsq(A, fs, rcond=None)
        assert np.max(np.abs(A @ b - fs)) < 1e-15
        for j, (mx, my) in enumerate(ms):
            n = mx + my
            got = b[j] * math.factorial(mx) * math.factorial(my) * cs2 ** n
            want = rho * ux ** mx * uy ** my + k * an.get((mx, my), 0.0)
            assert abs(got - want) < 1e-14, ((mx, my), got, want)
        # the equilibrium alone: coefficients rho u^m
        fe, _, _ = o.feq(rho, (ux, uy))
        b, *_ = np.linalg.lstsq(A, fe, rcond=None)
        assert np.max(np.abs(A @ b - fe)) < 1e-15
        for j, (mx, my) in enumerate(ms):
            got = b[j] * math.factorial(mx) * math.factorial(my) * cs2 ** (mx + my)
            assert abs(got - rho * ux ** mx * uy ** my) < 1e-14


def test_bgk_relaxation():
    o = Oracle("D2Q9", "BGK", nu_finest=0.1)
    f, fs = rr_case(o, 0.6)
    rho = f.sum()
    u = o.c[:, :2].T @ f / rho
    fe, _, _ = o.feq(rho, u)
    assert np.max(np.abs(fs - (f - (f - fe) / 0.6))) < 1e-16


def test_kinetic_sensor_bands():
    """Eqs. DeltaAvg / shock_function: alpha = 1 below 0.01, 1.05 on
    [0.01, 0.1), A on [0.1, 1), 1/tau above (tau_eff = tau alpha)."""
    A, tau = 1.5, 0.7
    o = Oracle("D2Q37", "DDF_POLY", T0=1.0, sensor_A=A, sensor_on=True, gamma=1.4)
    rho, u, T = 1.0, np.array([0.1, -0.05]), 0.9
    fe, ge, _ = o.feq(rho, u, T)
    # perturbations that keep rho, u and T (orthogonal to the moments)
    xi = o.c[:, :2].astype(float)
    xi2 = (xi ** 2).sum(1)
    basis = np.stack([np.ones(o.Q), xi[:, 0], xi[:, 1], xi2])
    d = rng.standard_normal(o.Q) * fe
    d = d - basis.T @ np.linalg.lstsq(basis.T, d, rcond=None)[0]
    for target, alpha in [(0.003, 1.0), (0.05, 1.05), (0.4, A), (2.5, 1.0 / tau)]:
        # scale the moment-free perturbation so that eps hits the target
        s = target / np.mean(np.abs(d) / np.abs(fe))
        f = fe + s * d
        fs, gs, _, eps = o.collide(tau, f, ge)
        assert abs(eps - np.mean(np.abs(f - fe) / np.abs(fe))) < 1e-12
        te = tau * alpha
        assert np.max(np.abs(fs - (f - (f - fe) / te))) < 1e-13, (target, alpha)
        assert np.max(np.abs(gs - ge)) < 1e-14  # g is already at equilibrium


def newton_residual(o, u, T, lam):
    xi = o.c[:, :2].astype(float)
    x, y = xi[:, 0], xi[:, 1]
    n2 = x * x + y * y
    mvec = np.stack([np.ones(o.Q), x, y, x * x, x * y, y * y, x * n2, y * n2])
    f = np.exp(-(1.0 + lam @ mvec))
    uu = u[0] ** 2 + u[1] ** 2
    # App. A.2: G^(0..3) with 2(E+T) = |u|^2 + 4T in 2-D
    M = np.array([1, u[0], u[1], u[0] ** 2 + T, u[0] * u[1], u[1] ** 2 + T,
                  u[0] * (uu + 4 * T), u[1] * (uu + 4 * T)])
    return mvec @ f - M


NEWTON_STATES = {
    "D2Q21": (0.65, [((0.3, -0.2), 0.65), ((1.43, 0.0), 0.65), ((0.0, 0.0), 0.9), ((0.5, 0.7), 0.5)]),
    "D2Q13": (0.35, [((0.3, -0.2), 0.35), ((0.8, 0.0), 0.35), ((0.0, 0.0), 0.5), ((0.3, 0.4), 0.3)]),
    "D2Q37": (1.0, [((0.3, -0.2), 1.0), ((2.0, 0.0), 1.0), ((0.0, 0.0), 1.3), ((0.9, 1.1), 0.8)]),
}


@pytest.mark.parametrize("name", list(NEWTON_STATES))
def test_newton_solves_constraints_and_symmetries(name):
    T0, states = NEWTON_STATES[name]
    o = Oracle(name, "DDF_NEWTON", T0=T0, gamma=1.4)
    for u, T in states:
        it, lam = o.newton(u, T)
        assert it >= 0
        assert np.max(np.abs(newton_residual(o, u, T, lam))) <= 1e-12
    # u = 0: every multiplier of an odd moment vanishes and xx == yy
    _, lam0 = o.newton((0.0, 0.0), 0.8)
    assert np.max(np.abs(lam0[[1, 2, 4, 6, 7]])) < 1e-12
    assert abs(lam0[3] - lam0[5]) < 1e-12
    # swapping x and y swaps the multipliers
    _, la = o.newton((0.4, -0.1), 0.7)
    _, lb = o.newton((-0.1, 0.4), 0.7)
    perm = [0, 2, 1, 5, 4, 3, 7, 6]
    assert np.max(np.abs(la[perm] - lb)) < 1e-10
    # the equilibrium scales with rho, the multipliers do not
    f1, _, l1 = o.feq(1.0, (0.4, 0.1), 0.7)
    f2, _, l2 = o.feq(3.0, (0.4, 0.1), 0.7)
    assert np.max(np.abs(3.0 * f1 - f2)) < 1e-14 and np.max(np.abs(l1 - l2)) < 1e-15


def test_newton_warm_start_iterations():
    """App. A / Sec. 3.2: ~10-12 iterations from lambda = 0, about one when
    warm-started from a nearby state."""
    o = Oracle("D2Q21", "DDF_NEWTON", T0=0.65, gamma=1.4)
    cold, lam = o.newton((0.3, 0.1), 0.65)
    assert 6 <= cold <= 15
    warm, _ = o.newton((0.3 + 1e-7, 0.1 - 1e-7), 0.65 + 1e-7, lam=lam)
    assert warm <= 2


def test_newton_rejects_unrealizable_state():
    """u_x^2 + T beyond max xi_x^2 = 9 cannot be matched by positive
    populations: the solver must report failure, not a value."""
    o = Oracle("D2Q21", "DDF_NEWTON", T0=0.65, gamma=1.4)
    it, _ = o.newton((2.5, 0.0), 3.0, max_it=60)
    assert it < 0


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_rr_trace_equilibration(name):
    """RR with trace equilibration (App. A.2, closing remark on the bulk
    relaxation): the trace of the second-order non-equilibrium tensor is
    relaxed with a relaxation time of one (it vanishes after collision) while
    its deviatoric part keeps the factor (1 - 1/tau); mass and momentum are
    conserved, and the kept third- and higher-order non-equilibrium moments
    follow from the filtered second-order tensor (pair-sum closed form).
    Every reference quantity is computed here from raw moments of the
    populations (second moment minus rho u u minus rho cs2 I), a route the
    oracle does not take (it projects f - f_eq on the Hermite basis).  A
    wrong sign or a wrong 1/D in the trace removal leaves a non-zero trace
    and fails."""
    o = Oracle(name, "RR", nu_finest=0.1, trace_eq=True)
    o_plain = Oracle(name, "RR", nu_finest=0.1)
    D = o.D
    xi = o.c[:, :D].astype(float)
    cs2 = o.cs2
    for tau in (0.62, 0.9, 1.7):
        k = 1.0 - 1.0 / tau
        for _ in range(4):
            rho = 0.9 + 0.2 * rng.random()
            u = 0.15 * (rng.random(D) - 0.5)
            fe, _, _ = o.feq(rho, u)
            # a bulk-heavy perturbation: isotropic plus random parts
            f = fe * (1.0 + 0.04 * (rng.random(o.Q) - 0.5) + 0.03 * ((xi ** 2).sum(1) - D * cs2))
            fs, _, _, _ = o.collide(tau, f)
            rho0 = f.sum()
            u0 = xi.T @ f / rho0
            assert abs(fs.sum() - rho0) < 1e-14
            assert np.max(np.abs(xi.T @ fs - rho0 * u0)) < 1e-15
            P = np.einsum("i,ia,ib->ab", f, xi, xi)
            aneq = P - rho0 * np.outer(u0, u0) - rho0 * cs2 * np.eye(D)
            assert abs(np.trace(aneq)) > 1e-4  # the case has a bulk part to remove
            dev = aneq - np.trace(aneq) / D * np.eye(D)
            Ps = np.einsum("i,ia,ib->ab", fs, xi, xi)
            aneq_s = Ps - rho0 * np.outer(u0, u0) - rho0 * cs2 * np.eye(D)
            assert abs(np.trace(aneq_s)) < 1e-14, np.trace(aneq_s)
            assert np.max(np.abs(aneq_s - k * dev)) < 1e-14
            # kept higher orders: the pair-sum closed form on the filtered tensor
            for m in itertools.product(range(3), repeat=D):
                tup = [d for d in range(D) for _ in range(m[d])]
                n = len(tup)
                if n < 3:
                    continue
                an = 0.0
                for p, q in itertools.combinations(range(n), 2):
                    pu = 1.0
                    for kk in range(n):
                        if kk not in (p, q):
                            pu *= u0[tup[kk]]
                    an += dev[tup[p], tup[q]] * pu
                aeq = rho0 * np.prod(u0 ** np.array(m))
                got = hermite_project(o, fs, m)
                assert abs(got - (aeq + k * an)) < 3e-15, (m, got, aeq + k * an)
            # without the flag the trace keeps the factor (1 - 1/tau)
            fp, _, _, _ = o_plain.collide(tau, f)
            Pp = np.einsum("i,ia,ib->ab", fp, xi, xi)
            tr_p = np.trace(Pp - rho0 * np.outer(u0, u0) - rho0 * cs2 * np.eye(D))
            assert abs(tr_p - k * np.trace(aneq)) < 1e-14
