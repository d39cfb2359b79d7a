"""Seeded synthetic workloads shaped like the paper's test cases.

This module only describes inputs: level masks, solid masks, face boundary
conditions, physical parameters and initial macroscopic fields.  It holds none
of the lattice Boltzmann arithmetic, so the HIP library and the CPU oracle can
both consume it.

Array convention: masks are numpy uint8 arrays of shape (Ey, Ex) in 2-D or
(Ez, Ey, Ex) in 3-D (x fastest in memory).  ``refine[l-1]`` has level l-1
resolution and marks the level l-1 cells that are refined to level >= l;
``solid[l]`` has level l resolution.

Workloads (coarse extents, levels ``0`` = coarsest):
  cavity   -- lid-driven cavity, D2Q9 BGK FP64 (Sec. 5.2 family)
  cylinder -- flow past a cylinder, D2Q9 RR FP32 (Sec. 5.3 family)
  sphere   -- flow past a sphere, D3Q27 RR FP32 / FP16 (Sec. 10 outlook case)
  sod      -- 1-D shock tube in 2-D, D2Q37 DDF (Sec. 6.1 family)
  airfoil  -- supersonic symmetric airfoil, D2Q21 numerical equilibrium
              (Sec. 6.3 family)
  shear    -- periodic doubly-refined shear-layer box used by tests
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea & Flood 2014), vectorised on uint64."""
    z = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def uniform_noise(seed: int, ids: np.ndarray, stream: int, amplitude: float) -> np.ndarray:
    """Uniform values in [-amplitude, amplitude) keyed by (seed, cell id, stream)."""
    key = (np.uint64(seed) << np.uint64(40)) ^ (np.uint64(stream) << np.uint64(36))
    with np.errstate(over="ignore"):
        bits = splitmix64(ids.astype(np.uint64) ^ key)
    u01 = (bits >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (2.0 * u01 - 1.0) * amplitude


@dataclasses.dataclass
class Mask:
    """A level mask restricted to a box: `data` (uint8, shape (ny, nx) or
    (nz, ny, nx)) covers cells [lo, lo + shape) of its level; every cell
    outside the box is 0."""
    data: np.ndarray
    lo: tuple

    @property
    def n(self):
        return tuple(reversed(self.data.shape))

    def dense(self, extent) -> np.ndarray:
        """full array over a level of extent (Ex, Ey[, Ez])."""
        out = np.zeros(tuple(reversed(tuple(extent))), np.uint8)
        sl = tuple(slice(self.lo[a], self.lo[a] + self.n[a]) for a in reversed(range(len(extent))))
        out[sl] = self.data
        return out


@dataclasses.dataclass
class Face:
    kind: str = "periodic"  # periodic | wall | moving_wall | neumann | equilibrium
    rho: float = 1.0
    u: tuple = (0.0, 0.0, 0.0)
    T: float = 0.0
    extrapolate_rho: bool = False
    sponge_sigma_max: float = 0.0
    sponge_width: float = 0.0


@dataclasses.dataclass
class Workload:
    name: str
    lattice: str
    collision: str
    dim: int
    ext: tuple
    n_levels: int
    refine: List[Mask]
    solid: List[Optional[Mask]]
    faces: List[Face]
    nu_finest: float
    steps: int
    T0: float = 0.0
    gamma: float = 1.4
    sensor_A: float = 1.5
    sensor_on: bool = False
    trace_eq: bool = False
    newton_tol: float = 1e-12
    newton_max_it: int = 100
    warm_start: bool = True
    # macroscopic initial state from (coords [n,3] int32, level [n] int8, ids)
    init: Callable = None
    # per-cell perturbation of the moving-wall velocity, (coords, level) ->
    # [3][n] in canonical order, or None
    inflow_noise: Optional[Callable] = None
    # optional host-side face schedule: step index -> {face: Face}
    schedule: Optional[Callable] = None
    storage: str = "fp64"

    def initial_moments(self, coords: np.ndarray, level: np.ndarray) -> np.ndarray:
        return self.init(np.asarray(coords), np.asarray(level))

    @property
    def n_mom(self) -> int:
        return 1 + self.dim + (1 if self.collision.startswith("DDF") else 0)


def _level_extent(ext, dim, level):
    return tuple(e << level for e in ext[:dim])


def _box_mask(ext, dim, level, lo, hi):
    """mask at level `level` of the cells inside the coarse-unit box [lo, hi)."""
    s = 1 << level
    lo_l = tuple(int(lo[a]) * s for a in range(dim))
    n_l = tuple((int(hi[a]) - int(lo[a])) * s for a in range(dim))
    return Mask(np.ones(tuple(reversed(n_l)), np.uint8), lo_l)


def _body_mask(ext, dim, level, lo, hi, inside):
    """mask at level `level` of the cells whose centre satisfies `inside`
    (a function of coarse-unit centre coordinates), searched in the
    coarse-unit bounding box [lo, hi)."""
    s = 1 << level
    E = _level_extent(ext, dim, level)
    a0 = [max(0, int(math.floor(lo[a] * s)) - 1) for a in range(dim)]
    a1 = [min(E[a], int(math.ceil(hi[a] * s)) + 1) for a in range(dim)]
    g = [(np.arange(a0[a], a1[a]) + 0.5) / s for a in range(dim)]
    if dim == 2:
        yy, xx = np.meshgrid(g[1], g[0], indexing="ij")
        m = inside(xx, yy)
    else:
        zz, yy, xx = np.meshgrid(g[2], g[1], g[0], indexing="ij")
        m = inside(xx, yy, zz)
    return Mask(m.astype(np.uint8), tuple(a0))


def _centre_coords(coords, level):
    return (coords.astype(np.float64) + 0.5) / (2.0 ** level.astype(np.float64))[:, None]


# --------------------------------------------------------------------------
# lid-driven cavity: D2Q9 BGK, two levels, top quarter refined (or one
# level and any weakly compressible lattice / collision, Sec. 5.2 and the
# uniform-grid performance runs)
# --------------------------------------------------------------------------
def cavity(n: int = 64, steps: int = 1000, lid: float = 0.1, Re: float = 100.0,
           refined_rows: Optional[int] = None, levels: int = 2, lattice: str = "D2Q9",
           collision: str = "BGK", storage: str = "fp64") -> Workload:
    dim, ext = 2, (n, n)
    rr = n // 4 if refined_rows is None else refined_rows
    refine = []
    if levels >= 2:
        refine.append(_box_mask(ext, dim, 0, (0, n - rr), (n, n)))
    nu0 = lid * n / Re                       # coarse-level viscosity
    nu_f = nu0 * (1 << (levels - 1))         # acoustic scaling, finest level
    faces = [Face("wall"), Face("wall"), Face("wall"),
             Face("moving_wall", u=(lid, 0.0, 0.0)), Face(), Face()]

    def init(coords, level):
        m = np.zeros((3, coords.shape[0]))
        m[0] = 1.0
        return m

    return Workload("cavity", lattice, collision, dim, ext, levels, refine,
                    [None] * levels, faces, nu_f, steps, init=init, storage=storage)


# --------------------------------------------------------------------------
# flow past a cylinder: D2Q9 RR, four levels of nested boxes
# --------------------------------------------------------------------------
def cylinder(scale: int = 1, steps: int = 2000, seed: int = 2, Ma: float = 0.2,
             Re: float = 150.0, storage: str = "fp32") -> Workload:
    """scale = 1 is the full 1024 x 512 coarse domain; scale = k divides every
    length by k (same structure)."""
    dim = 2
    ext = (1024 // scale, 512 // scale)
    boxes = [((64, 64), (1000, 448)), ((128, 128), (896, 384)), ((192, 192), (640, 320))]
    boxes = [(tuple(v // scale for v in lo), tuple(v // scale for v in hi)) for lo, hi in boxes]
    L = 4
    refine = [_box_mask(ext, dim, l, *boxes[l]) for l in range(L - 1)]
    cx, cy, radius = 256.0 / scale, 256.0 / scale, 20.0 / scale
    solid = [_body_mask(ext, dim, l, (cx - radius, cy - radius), (cx + radius, cy + radius),
                        lambda xx, yy: (xx - cx) ** 2 + (yy - cy) ** 2 <= radius * radius)
             for l in range(L)]
    uinf = Ma * math.sqrt(1.0 / 3.0)
    d_fine = 2 * radius * (1 << (L - 1))
    nu_f = uinf * d_fine / Re
    sp = Face("neumann", rho=1.0, sponge_sigma_max=0.1, sponge_width=128.0 / scale)
    faces = [Face("moving_wall", u=(uinf, 0.0, 0.0)), sp, sp, sp, Face(), Face()]

    def init(coords, level):
        m = np.zeros((3, coords.shape[0]))
        m[0] = 1.0
        m[1] = uinf
        return m

    def noise(coords, level):
        # a fixed perturbation of the inflow velocity per cell (only the
        # cells with a link across the inflow face use theirs)
        ids = np.arange(coords.shape[0], dtype=np.int64)
        du = np.zeros((3, coords.shape[0]))
        du[0] = uniform_noise(seed, ids, 0, 1e-4)
        du[1] = uniform_noise(seed, ids, 1, 1e-4)
        return du

    return Workload("cylinder", "D2Q9", "RR", dim, ext, L, refine, solid, faces,
                    nu_f, steps, init=init, storage=storage, inflow_noise=noise)


# --------------------------------------------------------------------------
# flow past a sphere: D3Q27 RR, three octree levels
# --------------------------------------------------------------------------
def sphere(scale: int = 1, steps: int = 500, seed: int = 3, Ma: float = 0.1,
           Re: float = 300.0, storage: str = "fp32") -> Workload:
    dim = 3
    ext = (512 // scale, 256 // scale, 256 // scale)
    boxes = [((80, 72, 72), (304, 184, 184)), ((104, 104, 104), (200, 152, 152))]
    boxes = [(tuple(v // scale for v in lo), tuple(v // scale for v in hi)) for lo, hi in boxes]
    L = 3
    refine = [_box_mask(ext, dim, l, *boxes[l]) for l in range(L - 1)]
    c0, radius = 128.0 / scale, 16.0 / scale
    solid = [_body_mask(ext, dim, l, (c0 - radius,) * 3, (c0 + radius,) * 3,
                        lambda xx, yy, zz: (xx - c0) ** 2 + (yy - c0) ** 2 + (zz - c0) ** 2 <= radius * radius)
             for l in range(L)]
    uinf = Ma * math.sqrt(1.0 / 3.0)
    nu_f = uinf * 2 * radius * (1 << (L - 1)) / Re
    nm = Face("neumann", rho=1.0)
    faces = [Face("moving_wall", u=(uinf, 0.0, 0.0)), nm, nm, nm, nm, nm]

    def init(coords, level):
        ids = np.arange(coords.shape[0], dtype=np.int64)
        m = np.zeros((4, coords.shape[0]))
        m[0] = 1.0
        m[1] = uinf + uniform_noise(seed, ids, 0, 1e-4)
        m[2] = uniform_noise(seed, ids, 1, 1e-4)
        m[3] = uniform_noise(seed, ids, 2, 1e-4)
        return m

    return Workload("sphere", "D3Q27", "RR", dim, ext, L, refine, solid, faces,
                    nu_f, steps, init=init, storage=storage)


# --------------------------------------------------------------------------
# Sod shock tube: D2Q37 DDF polynomial equilibrium, refined band (or any
# double-distribution lattice / equilibrium of the paper's Sec. 6.1)
# --------------------------------------------------------------------------
def sod(nx: int = 4096, ny: int = 8, steps: Optional[int] = None, theta: float = 0.65,
        sensor_A: float = 1.5, storage: str = "fp32", band: bool = True,
        lattice: str = "D2Q37", collision: str = "DDF_POLY", theta_at: str = "left") -> Workload:
    """(p, rho) = (1, 1) left and (0.1, 0.125) right, the paper's ratios;
    T = theta p / rho scaled so that the state named by theta_at ("left"
    or "right", the paper's reference state) has temperature theta."""
    dim, ext = 2, (nx, ny)
    L = 2 if band else 1
    refine = [_box_mask(ext, dim, 0, (nx // 4, 0), (3 * nx // 4, ny))] if band else []
    if steps is None:
        steps = int(0.2 * nx / math.sqrt(theta))
    nm = Face("neumann")
    faces = [nm, nm, Face("periodic"), Face("periodic"), Face(), Face()]

    def init(coords, level):
        xc = _centre_coords(coords, level)[:, 0]
        left = xc < nx / 2
        m = np.zeros((4, coords.shape[0]))
        m[0] = np.where(left, 1.0, 0.125)
        p = np.where(left, 1.0, 0.1)
        m[3] = theta * (p / m[0]) / (1.0 if theta_at == "left" else 0.8)
        return m

    return Workload("sod", lattice, collision, dim, ext, L, refine, [None] * L,
                    faces, 0.0, steps, T0=theta, gamma=1.4, sensor_A=sensor_A,
                    sensor_on=True, init=init, storage=storage)


# --------------------------------------------------------------------------
# supersonic airfoil: D2Q21 numerical equilibrium, three levels
# --------------------------------------------------------------------------
def naca_half_thickness(x: np.ndarray, t: float = 0.12) -> np.ndarray:
    """NACA four-digit symmetric thickness distribution (chord units)."""
    x = np.clip(x, 0.0, 1.0)
    return 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2
                      + 0.2843 * x ** 3 - 0.1015 * x ** 4)


def airfoil(scale: int = 1, steps: int = 1000, Ma: float = 1.5, Ma0: float = 1.0,
            ramp_steps: int = 200, Re: float = 1e4, T0: float = 0.65,
            storage: str = "fp32", warm_start: bool = True) -> Workload:
    dim = 2
    ext = (2048 // scale, 1024 // scale)
    boxes = [((320, 192), (1728, 832)), ((608, 384), (1280, 640))]
    boxes = [(tuple(v // scale for v in lo), tuple(v // scale for v in hi)) for lo, hi in boxes]
    L = 3
    refine = [_box_mask(ext, dim, l, *boxes[l]) for l in range(L - 1)]
    chord, le_x, le_y = 64.0 / scale, 704.0 / scale, 512.0 / scale
    def inside(xx, yy):
        xi = (xx - le_x) / chord
        return (xi >= 0.0) & (xi <= 1.0) & (np.abs(yy - le_y) / chord <= naca_half_thickness(xi))

    solid = [_body_mask(ext, dim, l, (le_x, le_y - 0.1 * chord), (le_x + chord, le_y + 0.1 * chord), inside)
             for l in range(L)]
    gamma = 1.4
    cs = math.sqrt(gamma * T0)
    uinf = Ma * cs
    nu_f = uinf * chord * (1 << (L - 1)) / Re

    def eq_face(m):
        return Face("equilibrium", rho=1.0, u=(m * cs, 0.0, 0.0), T=T0)

    faces = [eq_face(Ma0), Face("neumann"), eq_face(Ma0), eq_face(Ma0), Face(), Face()]

    def schedule(step):
        m = Ma0 + (Ma - Ma0) * min(1.0, step / float(ramp_steps)) if ramp_steps > 0 else Ma
        f = eq_face(m)
        return {0: f, 2: f, 3: f}

    def init(coords, level):
        m = np.zeros((4, coords.shape[0]))
        m[0] = 1.0
        m[1] = Ma0 * cs
        m[3] = T0
        return m

    return Workload("airfoil", "D2Q21", "DDF_NEWTON", dim, ext, L, refine, solid,
                    faces, nu_f, steps, T0=T0, gamma=gamma, sensor_A=1.35,
                    sensor_on=True, newton_tol=1e-12, newton_max_it=100,
                    warm_start=warm_start, init=init, schedule=schedule, storage=storage)


# --------------------------------------------------------------------------
# convected vortex with refinement patches that follow it (the adaptive runs
# of Sec. 8): periodic box, vortex carried along x
# --------------------------------------------------------------------------
def vortex(n: int = 64, levels: int = 3, lattice: str = "D2Q9", collision: str = "RR",
           u0: float = 0.05, eps: float = 0.02, radius: Optional[float] = None, nu_finest: float = 1e-3,
           steps: int = 64, storage: str = "fp64", T0: float = 1.0) -> Workload:
    """Gaussian vortex of radius R = n/16 (strength eps) at (n/4, n/2) in a
    uniform flow u0 along x.  `patch(t)` returns the refinement masks of
    nested square patches centred on where the vortex is after t coarse
    steps (half-widths 3R at level 0, 3R - 4 coarse cells deeper); the
    workload starts with patch(0)."""
    dim, ext = 2, (n, n)
    R = radius if radius is not None else n / 16.0
    x0, y0 = n / 4.0, n / 2.0
    ddf = collision.startswith("DDF")

    def patch(t):
        xc = x0 + u0 * t
        masks = []
        for l in range(levels - 1):
            h = 3.0 * R - 4.0 * l
            lo = (max(0, int(math.floor(xc - h))), max(0, int(math.floor(y0 - h))))
            hi = (min(n, int(math.ceil(xc + h))), min(n, int(math.ceil(y0 + h))))
            masks.append(_box_mask(ext, dim, l, lo, hi))
        return masks

    def init(coords, level):
        xc = _centre_coords(coords, level)
        dx, dy = (xc[:, 0] - x0) / R, (xc[:, 1] - y0) / R
        e = np.exp(-0.5 * (dx * dx + dy * dy))
        m = np.zeros((1 + dim + (1 if ddf else 0), coords.shape[0]))
        m[0] = 1.0 - 0.5 * eps * eps * e * e
        m[1] = u0 - eps * dy * e
        m[2] = eps * dx * e
        if ddf:
            m[3] = T0
        return m

    w = Workload("vortex", lattice, collision, dim, ext, levels, patch(0), [None] * levels,
                 [Face() for _ in range(6)], nu_finest, steps, T0=T0, init=init, storage=storage)
    w.patch = patch
    return w


# --------------------------------------------------------------------------
# periodic shear layers across refinement interfaces (tests)
# --------------------------------------------------------------------------
def shear(n: int = 32, levels: int = 2, lattice: str = "D2Q9", collision: str = "BGK",
          nu_finest: float = 0.02, steps: int = 10, kind: str = "dsl", u0: float = 0.05,
          band=None, seed: int = 7, storage: str = "fp64", T0: float = 1.0) -> Workload:
    """Periodic box.  kind="dsl": double shear layer of the paper's Sec. 5.1
    with a horizontal refinement band; kind="wave": decaying sinusoidal shear
    wave; kind="random": random smooth-ish perturbation.  `band` gives the
    refined rows of each level as fractions of n (nested).  Double
    distribution lattices start at the uniform temperature T0."""
    dim = 3 if lattice == "D3Q27" else 2
    ext = (n, n, n) if dim == 3 else (n, n)
    if band is None:
        band = [(0.5, 1.0), (0.625, 0.875), (0.6875, 0.8125)][: levels - 1]
    refine = []
    for l in range(levels - 1):
        lo = [0] * dim
        hi = list(ext)
        lo[1] = int(round(band[l][0] * n))
        hi[1] = int(round(band[l][1] * n))
        refine.append(_box_mask(ext, dim, l, tuple(lo), tuple(hi)))
    faces = [Face() for _ in range(6)]
    ddf = collision.startswith("DDF")

    def init(coords, level):
        xc = _centre_coords(coords, level)
        nm = 1 + dim + (1 if ddf else 0)
        m = np.zeros((nm, coords.shape[0]))
        m[0] = 1.0
        x, y = xc[:, 0] / n, xc[:, 1] / n
        if kind == "dsl":
            k, delta = 80.0, 0.05
            m[1] = np.where(y <= 0.5, u0 * np.tanh(k * (y - 0.25)), u0 * np.tanh(k * (0.75 - y)))
            m[2] = u0 * delta * np.sin(2.0 * np.pi * (x + 0.25))
        elif kind == "wave":
            m[1] = u0 * np.sin(2.0 * np.pi * y)
        else:
            ids = np.arange(coords.shape[0], dtype=np.int64)
            m[0] = 1.0 + uniform_noise(seed, ids, 3, 1e-2)
            for d in range(dim):
                m[1 + d] = uniform_noise(seed, ids, d, u0)
        if ddf:
            m[-1] = T0
        return m

    return Workload("shear", lattice, collision, dim, ext, levels, refine,
                    [None] * levels, faces, nu_finest, steps, T0=T0, init=init,
                    storage=storage)


# --------------------------------------------------------------------------
# training states of the multiplier surrogate
# --------------------------------------------------------------------------
def mlp_samples(n: int, seed: int = 5, rho=(0.2, 5.0), umax: float = 2.5, T=(0.5, 3.0)) -> np.ndarray:
    """n states (rho, u_x, u_y, T): rho and T uniform on their ranges, u
    uniform over the disc |u| <= umax (area-uniform radius)."""
    ids = np.arange(n, dtype=np.int64)
    a = [(uniform_noise(seed, ids, k, 1.0) + 1.0) * 0.5 for k in range(4)]
    r = umax * np.sqrt(a[1])
    th = 2.0 * np.pi * a[2]
    return np.stack([rho[0] + (rho[1] - rho[0]) * a[0], r * np.cos(th), r * np.sin(th),
                     T[0] + (T[1] - T[0]) * a[3]], axis=1)


REGISTRY = {
    "cavity": cavity,
    "cylinder": cylinder,
    "sphere": sphere,
    "sod": sod,
    "airfoil": airfoil,
    "shear": shear,
}
