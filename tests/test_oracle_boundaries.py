"""Closed-form pins of the oracle's boundary treatments that no flow field
with a known solution covers: the pressure sponge (Eq. relaxation_pressure:
the density that enters the equilibrium is relaxed towards the far field
before the collision) and the equilibrium (Dirichlet) faces of App. A.3,
with the density imposed or taken from the fluid next to the layer.

A fluid at rest with uniform density (and temperature) is at equilibrium,
and its equilibrium populations are proportional to the density.  One
collision of such a state therefore leaves every cell at the rest
equilibrium of a density known in closed form (boundary cells at the
face's equilibrium), and one pull streaming through the exported source
list gives every population after the step; the oracle must reproduce
them to rounding.  Longer runs check the fixed points: the sponge drives a
closed box to the far-field density, and a uniform flow that agrees with an
equilibrium inflow face and a Neumann outflow face stays uniform."""
import numpy as np
import pytest

from oracle.oracle import F_BC_EQ, F_BC_NEUMANN, F_SPONGE, Oracle
from paper_2504_04465_amd import workloads as W

CASES = [("D2Q9", "BGK"), ("D2Q9", "RR"), ("D2Q37", "DDF_POLY")]


def channel(lattice, collision, nx, ny, faces, nu=0.05):
    """one-level box, periodic along y, the given x faces"""
    w = W.shear(n=nx, levels=1, lattice=lattice, collision=collision, nu_finest=nu)
    w.ext = (nx, ny)
    w.faces = list(faces) + [W.Face() for _ in range(6 - len(faces))]
    return w


def uniform(rho, u, T, ddf):
    def init(coords, level):
        n = len(coords)
        m = [np.full(n, rho), np.full(n, u[0]), np.full(n, u[1])]
        if ddf:
            m.append(np.full(n, T))
        return np.vstack(m)
    return init


def pull_once(o, nbr, P):
    """populations after one pull streaming of the post-collision field
    P [n][Q]: source cell if any, own population where the source is
    outside an open face, own opposite population at a wall"""
    assert np.all(nbr >= -2), "no moving walls in these cases"
    f = np.empty_like(P)
    f[:, 0] = P[:, 0]
    for i in range(1, o.Q):
        v = nbr[:, i - 1]
        f[:, i] = np.where(v >= 0, P[np.maximum(v, 0), i], np.where(v == -1, P[:, i], P[:, o.opp[i]]))
    return f


@pytest.mark.parametrize("lattice,collision", CASES)
def test_sponge_one_step_closed_form(lattice, collision):
    nx, ny, width, smax, rho0, rinf, T = 24, 4, 7.0, 0.1, 1.0, 1.03, 1.0
    faces = [W.Face("wall", rho=rinf, sponge_sigma_max=smax, sponge_width=width), W.Face("wall")]
    w = channel(lattice, collision, nx, ny, faces)
    ddf = collision.startswith("DDF")
    w.init = uniform(rho0, (0.0, 0.0), T, ddf)
    o = Oracle.from_workload(w)
    o.init_workload(w)
    e = o.export()
    x = e["coords"][:, 0]
    # the paper's linear ramp of sigma, with the distance of the cell centre
    # to the face in place of the radius: sigma_max at the face, 0 from W on
    sigma = smax * np.clip(1.0 - (x + 0.5) / width, 0.0, 1.0)
    assert np.array_equal((e["flags"] & F_SPONGE) != 0, sigma > 0)
    rho_s = rho0 * (1.0 - sigma) + sigma * rinf
    # the relaxed density enters the equilibrium only: RR rebuilds the
    # populations from it; BGK and the DDF collision move 1/tau of the way
    tau = o.tau(0)
    rho_post = rho_s if collision == "RR" else rho0 - (rho0 - rho_s) / tau
    phi_f, phi_g, _ = o.feq(1.0, [0.0, 0.0], T)
    f_exp = pull_once(o, e["nbr"], rho_post[:, None] * phi_f[None, :])
    o.step(1)
    f, g, _ = o.state()
    assert np.max(np.abs(f - f_exp)) < 1e-14 * np.max(np.abs(f_exp))
    if ddf:
        g_exp = pull_once(o, e["nbr"], rho_post[:, None] * phi_g[None, :])
        assert np.max(np.abs(g - g_exp)) < 1e-14 * np.max(np.abs(g_exp))
    # a dropped or reversed sponge term would leave the density at rho0
    assert np.max(np.abs(o.moments()[0] - rho0)) > 1e-4


def test_sponge_drives_closed_box_to_far_field():
    """walls all round (mass would be conserved without the sponge): the
    sponge's only fixed point at rest is the far-field density"""
    nx, ny, rinf = 24, 4, 1.02
    faces = [W.Face("wall", rho=rinf, sponge_sigma_max=0.1, sponge_width=8.0), W.Face("wall")]
    w = channel("D2Q9", "RR", nx, ny, faces, nu=0.1)
    w.init = uniform(1.0, (0.0, 0.0), 0.0, False)
    o = Oracle.from_workload(w)
    o.init_workload(w)
    o.step(4000)
    m = o.moments()
    assert np.max(np.abs(m[0] - rinf)) < 1e-8
    assert np.max(np.abs(m[1:])) < 1e-9


@pytest.mark.parametrize("lattice,collision", [c for c in CASES if c[1] != "BGK"])
@pytest.mark.parametrize("extrapolate", [False, True])
def test_equilibrium_face_one_step(lattice, collision, extrapolate):
    nx, ny, rho0, T = 20, 4, 1.0, 1.0
    rb, ub, Tb = 1.05, (0.04, 0.01), 1.1
    ddf = collision.startswith("DDF")
    face = W.Face("equilibrium", rho=rb, u=(ub[0], ub[1], 0.0), T=Tb if ddf else 0.0, extrapolate_rho=extrapolate)
    w = channel(lattice, collision, nx, ny, [face, W.Face("neumann")])
    w.init = uniform(rho0, (0.0, 0.0), T, ddf)
    o = Oracle.from_workload(w)
    o.init_workload(w)
    e = o.export()
    eq = (e["flags"] & F_BC_EQ) != 0
    ne = (e["flags"] & F_BC_NEUMANN) != 0
    # B cells deep at each face
    assert eq.sum() == o.B * ny and ne.sum() == o.B * ny
    assert np.all(e["coords"][eq, 0] < o.B) and np.all(e["coords"][ne, 0] >= nx - o.B)
    # fluid and Neumann cells stay at rest; the inflow layer takes the
    # face's equilibrium, with the fluid's density when extrapolating
    phi_f, phi_g, _ = o.feq(1.0, [0.0, 0.0], T)
    fb, gb, _ = o.feq(rho0 if extrapolate else rb, ub, Tb if ddf else 0.0)
    Pf = np.tile(rho0 * phi_f, (o.n, 1))
    Pf[eq] = fb
    f_exp = pull_once(o, e["nbr"], Pf)
    o.step(1)
    f, g, _ = o.state()
    assert np.max(np.abs(f - f_exp)) < 1e-14 * np.max(np.abs(f_exp))
    if ddf:
        Pg = np.tile(rho0 * phi_g, (o.n, 1))
        Pg[eq] = gb
        g_exp = pull_once(o, e["nbr"], Pg)
        assert np.max(np.abs(g - g_exp)) < 1e-14 * np.max(np.abs(g_exp))
    # the inflow reaches the first fluid cells within the step
    m = o.moments()
    first = (e["coords"][:, 0] == o.B)
    assert np.all(m[1][first] > 1e-3)


@pytest.mark.parametrize("lattice,collision", [c for c in CASES if c[1] != "BGK"])
def test_uniform_flow_through_equilibrium_and_neumann_faces(lattice, collision):
    """inflow face at the state of the flow, Neumann outflow: nothing changes"""
    nx, ny, rho0, u0, T = 20, 4, 1.0, (0.05, -0.02), 1.0
    ddf = collision.startswith("DDF")
    face = W.Face("equilibrium", rho=rho0, u=(u0[0], u0[1], 0.0), T=T if ddf else 0.0)
    w = channel(lattice, collision, nx, ny, [face, W.Face("neumann")])
    w.init = uniform(rho0, u0, T, ddf)
    o = Oracle.from_workload(w)
    o.init_workload(w)
    o.step(200)
    m = o.moments()
    ref = [rho0, u0[0], u0[1]] + ([T] if ddf else [])
    for k, v in enumerate(ref):
        assert np.max(np.abs(m[k] - v)) < 1e-12, (k, np.max(np.abs(m[k] - v)))


def _walk_source(x, faces_in, E, B):
    """first fluid cell along the inward normal of every open face whose
    B-cell layer holds x: step inward one cell at a time until the cell
    leaves that face's layer (corners move along both normals)"""
    q = list(x)
    for fc in faces_in:
        a, hi = fc // 2, fc & 1
        while (q[a] >= E[a] - B) if hi else (q[a] < B):
            q[a] += -1 if hi else 1
    return tuple(q)


@pytest.mark.parametrize("lattice,collision", [("D2Q9", "BGK"), ("D2Q21", "RR"), ("D2Q37", "DDF_POLY")])
def test_neumann_one_step_non_uniform_closed_form(lattice, collision):
    """Neumann faces on all four sides of a non-uniform field (App. A.3):
    after one step every population equals the post-collision population of
    its pull source, where a boundary cell's post-collision populations are
    those of the first fluid cell along the inward normal (both normals at a
    corner).  The state is at equilibrium, so a collision leaves it
    unchanged and f* = f_eq at each cell's own moments.  The sources and the
    streaming are recomputed here from coordinates alone (no exported
    neighbour or source list); a source one cell off, or a corner that is
    not clamped along both normals, changes the boundary values."""
    nx, ny = 14, 12
    ddf = collision.startswith("DDF")
    w = channel(lattice, collision, nx, ny, [W.Face("neumann"), W.Face("neumann"),
                                              W.Face("neumann"), W.Face("neumann")])
    r = np.random.default_rng(11)

    def init(coords, level):
        x = coords[:, 0] + 0.5
        y = coords[:, 1] + 0.5
        n = len(coords)
        rho = 1.0 + 0.08 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny) + 0.02 * r.random(n)
        m = [rho, 0.03 * np.cos(2 * np.pi * y / ny) + 0.01 * r.random(n), 0.02 * np.sin(2 * np.pi * x / nx)]
        if ddf:
            m.append(1.0 + 0.05 * r.random(n))
        return np.vstack(m)

    w.init = init
    o = Oracle.from_workload(w)
    e = o.export()
    coords = e["coords"][:, :2]
    m0 = init(coords, e["level"])
    o.init(m0)
    B, Q = o.B, o.Q
    index = {tuple(int(v) for v in coords[c]): c for c in range(o.n)}
    # post-collision state: the equilibrium of every cell's own moments
    Pf = np.zeros((o.n, Q))
    Pg = np.zeros((o.n, Q)) if ddf else None
    for c in range(o.n):
        fe, ge, _ = o.feq(m0[0, c], m0[1:3, c], m0[3, c] if ddf else 0.0)
        Pf[c] = fe
        if ddf:
            Pg[c] = ge
    E = (nx, ny)
    src = np.arange(o.n)
    for c in range(o.n):
        x = tuple(int(v) for v in coords[c])
        faces_in = [fc for fc in range(4) if ((x[fc // 2] >= E[fc // 2] - B) if fc & 1 else (x[fc // 2] < B))]
        if faces_in:
            q = _walk_source(x, faces_in, E, B)
            src[c] = index[q]
            assert e["flags"][c] & F_BC_NEUMANN
        else:
            assert not e["flags"][c] & (F_BC_NEUMANN | F_BC_EQ)
    Pf = Pf[src]
    if ddf:
        Pg = Pg[src]
    # pull streaming by coordinates; a source outside an open face keeps
    # the cell's own post-collision population
    f_exp = np.empty_like(Pf)
    g_exp = np.empty_like(Pf) if ddf else None
    for c in range(o.n):
        x = coords[c]
        for i in range(Q):
            q = (int(x[0]) - int(o.c[i][0]), int(x[1]) - int(o.c[i][1]))
            s = index.get(q, c)
            f_exp[c, i] = Pf[s, i]
            if ddf:
                g_exp[c, i] = Pg[s, i]
    o.step(1)
    f, g, _ = o.state()
    assert np.max(np.abs(f - f_exp)) < 1e-14 * np.max(np.abs(f_exp))
    if ddf:
        assert np.max(np.abs(g - g_exp)) < 1e-14 * np.max(np.abs(g_exp))
    # the case discriminates: a boundary cell's copied state differs from
    # the equilibrium of its own moments
    bc = np.nonzero(src != np.arange(o.n))[0]
    feq_own = np.array([o.feq(m0[0, c], m0[1:3, c], m0[3, c] if ddf else 0.0)[0] for c in bc])
    assert np.min(np.max(np.abs(Pf[bc] - feq_own), axis=1)) > 1e-5


def test_moving_wall_inflow_noise_one_step():
    """Ladd's moving wall (wall density 1) with a per-cell perturbation of
    the wall velocity (the cylinder's inflow noise): from a fluid at rest
    (post-collision state w_i), after one step every population that crosses
    the moving face equals w_opp + 2 w_i xi_i . (u_w + du_c) / cs2, every
    population that crosses the resting wall w_opp, and every other one w_i;
    the perturbation of other cells plays no part.  A dropped or reversed
    perturbation fails."""
    nx, ny = 8, 6
    uw = np.array([0.05, 0.01, 0.0])
    w = channel("D2Q9", "BGK", nx, ny, [W.Face("moving_wall", u=tuple(uw)), W.Face("wall")])
    w.init = uniform(1.0, (0.0, 0.0), 0.0, False)
    o = Oracle.from_workload(w)
    o.init_workload(w)
    e = o.export()
    r = np.random.default_rng(3)
    du = np.zeros((3, o.n))
    du[:2] = 1e-3 * (2 * r.random((2, o.n)) - 1)
    o.set_inflow_noise(du)
    o.step(1)
    f, _, _ = o.state()
    x = e["coords"][:, 0]
    exp = np.tile(o.w, (o.n, 1))
    for i in range(1, o.Q):
        j = o.opp[i]
        src = x - o.c[i][0]
        left = src < 0
        right = src >= nx
        cu = o.c[i][0] * (uw[0] + du[0]) + o.c[i][1] * (uw[1] + du[1])
        exp[left, i] = o.w[j] + 2 * o.w[i] * cu[left] / o.cs2
        exp[right, i] = o.w[j]
    assert np.max(np.abs(f - exp)) < 1e-15
    # the perturbation matters at the size it is given
    o2 = Oracle.from_workload(w)
    o2.init_workload(w)
    o2.step(1)
    f2, _, _ = o2.state()
    assert np.max(np.abs(f - f2)) > 1e-4
