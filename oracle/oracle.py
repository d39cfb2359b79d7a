"""ctypes wrapper of the plain FP64 CPU oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

LATTICES = {"D2Q9": 0, "D3Q27": 1, "D2Q21": 2, "D2Q37": 3, "D2Q13": 4}
COLLISIONS = {"BGK": 0, "RR": 1, "DDF_POLY": 2, "DDF_NEWTON": 3}
BC_KINDS = {"periodic": 0, "wall": 1, "moving_wall": 2, "neumann": 3, "equilibrium": 4}
NONE, SOLID = -1, -2
F_COARSE_GHOST, F_FINE_GHOST, F_BC_NEUMANN, F_BC_EQ, F_SPONGE = 1, 2, 4, 8, 16


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, optional OpenMP)."""
    src = os.path.join(HERE, "lbm_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Face(C.Structure):
    _fields_ = [("kind", C.c_int), ("rho", C.c_double), ("u", C.c_double * 3), ("T", C.c_double),
                ("extrapolate_rho", C.c_int), ("sponge_sigma_max", C.c_double),
                ("sponge_width", C.c_double)]


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("collision", C.c_int), ("nu_finest", C.c_double),
                ("T0", C.c_double), ("gamma", C.c_double), ("sensor_A", C.c_double),
                ("sensor_on", C.c_int), ("trace_eq", C.c_int), ("newton_tol", C.c_double),
                ("newton_max_it", C.c_int), ("warm_start", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
        L.ol_create.restype = vp
        L.ol_create.argtypes = [C.POINTER(Params)]
        L.ol_destroy.argtypes = [vp]
        L.ol_error.restype = C.c_char_p
        L.ol_error.argtypes = [vp]
        L.ol_lattice.argtypes = [vp] + [C.c_void_p] * 7
        L.ol_grid.argtypes = [vp, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ol_n_cells.restype = i64
        L.ol_n_cells.argtypes = [vp]
        L.ol_n_ghosts.restype = i64
        L.ol_n_ghosts.argtypes = [vp]
        L.ol_level_counts.argtypes = [vp, C.c_void_p]
        L.ol_export.argtypes = [vp] + [C.c_void_p] * 6
        L.ol_init.argtypes = [vp, C.c_void_p]
        L.ol_step.argtypes = [vp, i64]
        L.ol_moments.argtypes = [vp, C.c_void_p]
        L.ol_sums.argtypes = [vp, C.c_void_p]
        L.ol_kinetic_energy.argtypes = [vp, C.c_void_p]
        L.ol_set_face.argtypes = [vp, C.c_int, C.POINTER(Face)]
        L.ol_set_inflow_noise.argtypes = [vp, C.c_void_p]
        L.ol_counters.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ol_get_state.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ol_set_state.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ol_get_sync_state.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ol_sensor.argtypes = [vp, C.c_void_p]
        L.ol_feq.argtypes = [vp, C.c_double, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ol_collide.argtypes = [vp, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]
        L.ol_newton.argtypes = [vp, C.c_void_p, C.c_double, C.c_void_p, C.c_double, C.c_int]
        L.ol_tau.restype = C.c_double
        L.ol_tau.argtypes = [vp, C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_face(f) -> Face:
    out = Face()
    out.kind = BC_KINDS[f.kind]
    out.rho = f.rho
    for k in range(3):
        out.u[k] = f.u[k] if k < len(f.u) else 0.0
    out.T = f.T
    out.extrapolate_rho = int(f.extrapolate_rho)
    out.sponge_sigma_max = f.sponge_sigma_max
    out.sponge_width = f.sponge_width
    return out


class Oracle:
    """One oracle simulation.  `lattice`/`collision` are names such as
    "D2Q9"/"RR"; the remaining keywords mirror the C parameter block."""

    def __init__(self, lattice: str, collision: str, nu_finest: float = 0.0, T0: float = 0.0,
                 gamma: float = 1.4, sensor_A: float = 1.5, sensor_on: bool = False,
                 trace_eq: bool = False, newton_tol: float = 1e-12, newton_max_it: int = 100,
                 warm_start: bool = True):
        p = Params(LATTICES[lattice], COLLISIONS[collision], nu_finest, T0, gamma, sensor_A,
                   int(sensor_on), int(trace_eq), newton_tol, newton_max_it, int(warm_start))
        self._L = lib()
        self.h = self._L.ol_create(C.byref(p))
        if not self.h:
            raise ValueError(f"oracle rejected {lattice}/{collision}")
        self.lattice, self.collision = lattice, collision
        D, Q, B = C.c_int(), C.c_int(), C.c_int()
        cs2 = C.c_double()
        c = np.zeros(37 * 3, np.int32)
        w = np.zeros(37)
        opp = np.zeros(37, np.int32)
        self._L.ol_lattice(self.h, C.byref(D), C.byref(Q), C.byref(B), _ptr(c), _ptr(w),
                           C.byref(cs2), _ptr(opp))
        self.D, self.Q, self.B, self.cs2 = D.value, Q.value, B.value, cs2.value
        self.c = c[: 3 * self.Q].reshape(self.Q, 3).copy()
        self.w = w[: self.Q].copy()
        self.opp = opp[: self.Q].copy()
        self.ddf = collision.startswith("DDF")

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(nu_finest=w.nu_finest, T0=w.T0, gamma=w.gamma, sensor_A=w.sensor_A,
                  sensor_on=w.sensor_on, trace_eq=w.trace_eq, newton_tol=w.newton_tol,
                  newton_max_it=w.newton_max_it, warm_start=w.warm_start)
        kw.update(over)
        o = cls(w.lattice, w.collision, **kw)
        o.grid(w.dim, w.ext, w.n_levels, w.refine, w.solid, w.faces)
        return o

    def __del__(self):
        if getattr(self, "h", None):
            self._L.ol_destroy(self.h)
            self.h = None

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}: {self._L.ol_error(self.h).decode()}")

    def grid(self, dim, ext, n_levels, refine, solid, faces):
        """refine[l] / solid[l]: dense uint8 arrays of level l (shape (Ey, Ex)
        or (Ez, Ey, Ex)), or window objects with a dense(extent) method."""
        e = np.array(list(ext) + [1] * (3 - len(ext)), np.int32)

        def dense(m, level):
            if m is None:
                return None
            extent = tuple(int(x) << level for x in ext[:dim])
            if hasattr(m, "dense"):
                return m.dense(extent)
            return np.ascontiguousarray(m, dtype=np.uint8)

        self._keep = [dense(r, l) for l, r in enumerate(refine)]
        rp = (C.c_void_p * max(1, len(self._keep)))(*[_ptr(a) for a in self._keep])
        sp = None
        if solid is not None and any(s is not None for s in solid):
            sol = []
            for l in range(n_levels):
                s = dense(solid[l], l) if l < len(solid) else None
                if s is None:
                    s = np.zeros(tuple(int(x) << l for x in ext[:dim])[::-1], np.uint8)
                sol.append(s)
            self._keep_s = sol
            sp = (C.c_void_p * len(sol))(*[_ptr(a) for a in sol])
        fa = (Face * 6)(*[make_face(f) for f in faces])
        self._check(self._L.ol_grid(self.h, dim, _ptr(e), n_levels, rp, sp, fa))
        self._ext, self._faces = tuple(ext), list(faces)
        self.n = self._L.ol_n_cells(self.h)
        self.n_levels = n_levels
        self.dim = dim

    def level_counts(self):
        out = np.zeros(self.n_levels, np.int64)
        self._check(self._L.ol_level_counts(self.h, _ptr(out)))
        return out

    def export(self):
        n, Q = self.n, self.Q
        ng = self._L.ol_n_ghosts(self.h)
        d = dict(coords=np.zeros((n, 3), np.int32), level=np.zeros(n, np.int8),
                 flags=np.zeros(n, np.uint8), nbr=np.zeros((n, Q - 1), np.int32),
                 child=np.zeros((max(ng, 0), 1 << self.D), np.int32),
                 bc_src=np.zeros(n, np.int32))
        self._check(self._L.ol_export(self.h, _ptr(d["coords"]), _ptr(d["level"]), _ptr(d["flags"]),
                                      _ptr(d["nbr"]), _ptr(d["child"]), _ptr(d["bc_src"])))
        return d

    def init(self, moments):
        m = np.ascontiguousarray(moments, dtype=np.float64)
        self._check(self._L.ol_init(self.h, _ptr(m)))

    def init_workload(self, w):
        e = self.export()
        self.init(w.initial_moments(e["coords"], e["level"]))
        if getattr(w, "inflow_noise", None) is not None:
            self.set_inflow_noise(w.inflow_noise(e["coords"], e["level"]))

    def step(self, n=1):
        self._check(self._L.ol_step(self.h, n))

    def set_face(self, k, face):
        f = make_face(face)
        self._check(self._L.ol_set_face(self.h, k, C.byref(f)))

    def moments(self):
        nm = 1 + self.D + (1 if self.ddf else 0)
        out = np.zeros((nm, self.n))
        self._check(self._L.ol_moments(self.h, _ptr(out)))
        return out

    def sums(self):
        out = np.zeros(2 + self.D)
        self._check(self._L.ol_sums(self.h, _ptr(out)))
        return out

    def set_inflow_noise(self, du):
        """du [3][n] (canonical order) added to the moving-wall velocity seen
        by each cell; None removes it"""
        if du is None:
            self._check(self._L.ol_set_inflow_noise(self.h, None))
            return
        d = np.ascontiguousarray(du, dtype=np.float64)
        assert d.shape == (3, self.n)
        self._check(self._L.ol_set_inflow_noise(self.h, _ptr(d)))

    def kinetic_energy(self):
        out = C.c_double()
        self._check(self._L.ol_kinetic_energy(self.h, C.byref(out)))
        return out.value

    def counters(self):
        upd = np.zeros(8, np.int64)
        it, calls = C.c_int64(), C.c_int64()
        self._L.ol_counters(self.h, _ptr(upd), C.byref(it), C.byref(calls))
        return upd[: self.n_levels], it.value, calls.value

    def state(self):
        f = np.zeros((self.n, self.Q))
        g = np.zeros((self.n, self.Q)) if self.ddf else None
        lam = np.zeros((self.n, 8))
        self._check(self._L.ol_get_state(self.h, _ptr(f), _ptr(g), _ptr(lam)))
        return f, g, lam

    def sync_state(self):
        """state with every coarse ghost's unknown populations coalesced"""
        f = np.zeros((self.n, self.Q))
        g = np.zeros((self.n, self.Q)) if self.ddf else None
        lam = np.zeros((self.n, 8))
        self._check(self._L.ol_get_sync_state(self.h, _ptr(f), _ptr(g), _ptr(lam)))
        return f, g, lam

    def sensor(self):
        """kinetic sensor eps per cell (Eq. DeltaAvg), NaN for fine ghosts"""
        out = np.zeros(self.n)
        self._check(self._L.ol_sensor(self.h, _ptr(out)))
        return out

    def set_state(self, f, g=None, lam=None):
        """pre-collision populations [n][Q] (g likewise, multipliers [n][8])"""
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
        self._check(self._L.ol_set_state(self.h, _ptr(f), _ptr(g), _ptr(lam)))

    def tau(self, level):
        return self._L.ol_tau(self.h, level)

    # single-cell helpers --------------------------------------------------
    def feq(self, rho, u, T=0.0, lam=None):
        u3 = np.zeros(3)
        u3[: len(u)] = u
        fe = np.zeros(self.Q)
        ge = np.zeros(self.Q)
        lm = np.zeros(8) if lam is None else np.array(lam, dtype=np.float64)
        self._check(self._L.ol_feq(self.h, rho, _ptr(u3), T, _ptr(fe), _ptr(ge), _ptr(lm)))
        return fe, (ge if self.ddf else None), lm

    def collide(self, tau, f, g=None, lam=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        fs = np.zeros(self.Q)
        gs = np.zeros(self.Q)
        lm = np.zeros(8) if lam is None else np.array(lam, dtype=np.float64)
        eps = C.c_double(-1.0)
        self._check(self._L.ol_collide(self.h, tau, _ptr(f), _ptr(g), _ptr(fs), _ptr(gs), _ptr(lm),
                                       C.byref(eps)))
        return fs, (gs if self.ddf else None), lm, eps.value

    def newton(self, u, T, lam=None, tol=1e-12, max_it=100):
        u3 = np.zeros(3)
        u3[: len(u)] = u
        lm = np.zeros(8) if lam is None else np.array(lam, dtype=np.float64)
        it = self._L.ol_newton(self.h, _ptr(u3), T, _ptr(lm), tol, max_it)
        return it, lm
