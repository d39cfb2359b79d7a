"""Thin Python binding of liblbm.so (C-ABI declared in include/lbm.h).

Argument marshalling only: every step of the update runs in the HIP library.
PyTorch supplies the device memory (caching allocator) and the stream.  There
is no fallback: if liblbm.so is missing or fails to load, this module raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# LBM_LIB_PATH selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("LBM_LIB_PATH", os.path.join(PKG, "liblbm.so"))

LATTICES = {"D2Q9": 0, "D3Q27": 1, "D2Q21": 2, "D2Q37": 3, "D2Q13": 4}
LATTICE_Q = {"D2Q9": 9, "D3Q27": 27, "D2Q21": 21, "D2Q37": 37, "D2Q13": 13}
COLLISIONS = {"BGK": 0, "RR": 1, "DDF_POLY": 2, "DDF_NEWTON": 3, "DDF_MLP": 4, "DDF_MLP_NEWTON": 5}
STORAGE = {"fp64": 0, "fp32": 1, "fp16": 2}
BC_KINDS = {"periodic": 0, "wall": 1, "moving_wall": 2, "neumann": 3, "equilibrium": 4}
STATUS = {0: "LBM_OK", -1: "LBM_E_ARG", -2: "LBM_E_MASK", -3: "LBM_E_NOMEM", -4: "LBM_E_DEVICE",
          -5: "LBM_E_STATE", -6: "LBM_E_NUMERIC", -7: "LBM_E_UNSUPPORTED"}

# every entry point declared in include/lbm.h
EXPORTS = ["lbm_create", "lbm_grid_build", "lbm_grid_info", "lbm_layout_info", "lbm_layout_export",
           "lbm_grid_export", "lbm_init",
           "lbm_step", "lbm_set_face_bc", "lbm_set_graphs", "lbm_moments", "lbm_moments_device", "lbm_stats_get",
           "lbm_sums_device", "lbm_set_level_fusion", "lbm_set_inflow_noise", "lbm_set_device_build",
           "lbm_sync", "lbm_profile_enable", "lbm_profile_read", "lbm_get_state", "lbm_get_cells", "lbm_set_state",
           "lbm_remesh", "lbm_sensor",
           "lbm_last_error", "lbm_destroy", "lbm_mlp_set_weights", "lbm_mlp_get_weights",
           "lbm_mlp_label", "lbm_mlp_predict", "lbm_mlp_grad", "lbm_mlp_train"]
MLP_PARAMS = 9176


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("collision", C.c_int), ("storage", C.c_int),
                ("nu_finest", C.c_double), ("T0", C.c_double), ("gamma", C.c_double),
                ("sensor_A", C.c_double), ("sensor_on", C.c_int), ("trace_equilibration", C.c_int),
                ("newton_tol", C.c_double), ("fallback_tol", C.c_double), ("newton_max_it", C.c_int),
                ("lambda_warm_start", C.c_int), ("host_only", C.c_int), ("in_place", C.c_int)]


class FaceBC(C.Structure):
    _fields_ = [("kind", C.c_int), ("rho", C.c_double), ("u", C.c_double * 3), ("T", C.c_double),
                ("extrapolate_rho", C.c_int), ("sponge_sigma_max", C.c_double),
                ("sponge_width", C.c_double)]


class MaskC(C.Structure):
    _fields_ = [("data", C.c_void_p), ("lo", C.c_int32 * 3), ("n", C.c_int32 * 3)]


class Stats(C.Structure):
    _fields_ = [("mass", C.c_double), ("momentum", C.c_double * 3), ("energy", C.c_double),
                ("kinetic_energy", C.c_double),
                ("updates", C.c_int64 * 8), ("newton_calls", C.c_int64),
                ("newton_iterations", C.c_int64), ("newton_failures", C.c_int64),
                ("mlp_fallbacks", C.c_int64), ("nonfinite_cells", C.c_int64),
                ("coarse_steps", C.c_int64), ("newton_hist", C.c_int64 * 16)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    """Load liblbm.so (built by paper_2504_04465_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        # load torch first: liblbm.so shares torch's HIP runtime
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2504_04465_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        L.lbm_create.argtypes = [C.POINTER(Params), ALLOC_FN, FREE_FN, vp, vp, C.POINTER(vp)]
        L.lbm_grid_build.argtypes = [vp, C.c_int, vp, C.c_int, vp, vp, vp]
        L.lbm_grid_info.argtypes = [vp, vp, vp, vp, vp]
        L.lbm_layout_info.argtypes = [vp, vp, vp, vp, vp]
        L.lbm_layout_export.argtypes = [vp] * 6
        L.lbm_grid_export.argtypes = [vp] + [vp] * 6
        L.lbm_init.argtypes = [vp, vp]
        L.lbm_step.argtypes = [vp, i64]
        L.lbm_set_face_bc.argtypes = [vp, C.c_int, C.POINTER(FaceBC)]
        L.lbm_set_graphs.argtypes = [vp, C.c_int]
        L.lbm_set_level_fusion.argtypes = [vp, C.c_int]
        L.lbm_set_device_build.argtypes = [vp, C.c_int]
        L.lbm_set_inflow_noise.argtypes = [vp, vp]
        L.lbm_moments.argtypes = [vp, vp]
        L.lbm_moments_device.argtypes = [vp, vp]
        L.lbm_stats_get.argtypes = [vp, C.POINTER(Stats)]
        L.lbm_sums_device.argtypes = [vp, vp]
        L.lbm_sync.argtypes = [vp]
        L.lbm_profile_enable.argtypes = [vp, C.c_int]
        L.lbm_profile_read.argtypes = [vp, C.c_int, vp, vp, vp]
        L.lbm_get_state.argtypes = [vp, vp, vp, vp]
        L.lbm_set_state.argtypes = [vp, vp, vp, vp]
        L.lbm_remesh.argtypes = [vp, vp, vp]
        L.lbm_sensor.argtypes = [vp, vp]
        L.lbm_get_cells.argtypes = [vp, vp, i64, vp, vp, vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_last_error.argtypes = [vp]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_mlp_set_weights.argtypes = [vp, vp, i64]
        L.lbm_mlp_get_weights.argtypes = [vp, vp, i64]
        L.lbm_mlp_label.argtypes = [vp, vp, i64, vp, vp, vp]
        L.lbm_mlp_predict.argtypes = [vp, vp, i64, vp]
        L.lbm_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp]
        L.lbm_mlp_train.argtypes = [vp, vp, vp, i64, C.c_int, C.c_int, C.c_double, C.c_uint64, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def face_struct(f) -> FaceBC:
    out = FaceBC()
    out.kind = BC_KINDS[f.kind]
    out.rho = f.rho
    for k in range(3):
        out.u[k] = f.u[k] if k < len(f.u) else 0.0
    out.T = f.T
    out.extrapolate_rho = int(f.extrapolate_rho)
    out.sponge_sigma_max = f.sponge_sigma_max
    out.sponge_width = f.sponge_width
    return out


def equivalent_fine_cells(n_per_level) -> float:
    """sum_l n_l / 2^(L-1-l): cells weighted by their update frequency
    relative to the finest level (Sec. 7.5)."""
    L = len(n_per_level)
    return float(sum(n / float(1 << (L - 1 - l)) for l, n in enumerate(n_per_level)))


class _TorchAlloc:
    """Device allocations from PyTorch's caching allocator on one stream."""

    def __init__(self, device, stream):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, size, _ctx):
        return self.torch.cuda.caching_allocator_alloc(int(size), self.device, self.stream)

    def _free(self, ptr, _ctx):
        self.torch.cuda.caching_allocator_delete(ptr)


# contexts still open at interpreter exit are destroyed while torch's
# allocator (which owns their device memory) is still usable
_LIVE: "weakref.WeakSet[LBM]" = weakref.WeakSet()


@atexit.register
def _close_all():
    for ctx in list(_LIVE):
        ctx.close()


class LBM:
    """One refined-grid lattice Boltzmann simulation in liblbm.so."""

    def __init__(self, lattice: str, collision: str, storage: str = "fp64", nu_finest: float = 0.0,
                 T0: float = 0.0, gamma: float = 1.4, sensor_A: float = 1.5, sensor_on: bool = False,
                 trace_eq: bool = False, newton_tol: float = 1e-12, fallback_tol: float = 1e-10,
                 newton_max_it: int = 100, warm_start: bool = True, host_only: bool = False,
                 in_place: bool = False, device: int = 0, stream=None):
        self._L = lib()
        p = Params(LATTICES[lattice], COLLISIONS[collision], STORAGE[storage], nu_finest, T0, gamma,
                   sensor_A, int(sensor_on), int(trace_eq), newton_tol, fallback_tol, newton_max_it,
                   int(warm_start), int(host_only), int(in_place))
        self.lattice, self.collision, self.storage = lattice, collision, storage
        self.ddf = collision.startswith("DDF")
        self.host_only = host_only
        self._alloc = None
        stream_ptr = None
        alloc_cb, free_cb = ALLOC_FN(), FREE_FN()
        if not host_only:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible: liblbm.so needs a device (or host_only=True)")
            torch.cuda.set_device(device)
            # a stream of the context's own (default priority): graph capture
            # needs a stream other than the null stream
            self.torch_stream = stream if stream is not None else torch.cuda.Stream(device)
            stream_ptr = self.torch_stream.cuda_stream
            self._alloc = _TorchAlloc(device, stream_ptr)
            alloc_cb, free_cb = self._alloc.alloc_cb, self._alloc.free_cb
        h = C.c_void_p()
        rc = self._L.lbm_create(C.byref(p), alloc_cb, free_cb, None, stream_ptr, C.byref(h))
        if rc != 0:
            raise LbmError(rc, f"lbm_create rejected {lattice}/{collision}/{storage}")
        self.h = h
        _LIVE.add(self)

    @classmethod
    def from_workload(cls, w, storage=None, host_only=False, **over):
        kw = dict(nu_finest=w.nu_finest, T0=w.T0, gamma=w.gamma, sensor_A=w.sensor_A,
                  sensor_on=w.sensor_on, trace_eq=w.trace_eq, newton_tol=w.newton_tol,
                  newton_max_it=w.newton_max_it, warm_start=w.warm_start)
        kw.update(over)
        s = cls(w.lattice, w.collision, storage or w.storage, host_only=host_only, **kw)
        s.grid(w.dim, w.ext, w.n_levels, w.refine, w.solid, w.faces)
        return s

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "h", None):
            self._L.lbm_destroy(self.h)
            self.h = None
            _LIVE.discard(self)

    def _check(self, rc, what=""):
        if rc != 0:
            raise LbmError(rc, f"{what}: {self._L.lbm_last_error(self.h).decode()}")

    # ---- grid ----------------------------------------------------------
    def grid(self, dim, ext, n_levels, refine, solid, faces):
        """refine[l] / solid[l] are window masks (objects with .data and .lo,
        data shaped (ny, nx) or (nz, ny, nx)) or None."""
        self.dim, self.n_levels = dim, n_levels
        e = np.array(list(ext) + [1] * (3 - len(ext)), np.int32)
        ra, sa, keep = self._masks(refine, solid, n_levels)
        fa = (FaceBC * 6)(*[face_struct(f) for f in faces])
        self._check(self._L.lbm_grid_build(self.h, dim, _ptr(e), n_levels, C.cast(ra, C.c_void_p),
                                           None if sa is None else C.cast(sa, C.c_void_p),
                                           C.cast(fa, C.c_void_p)), "lbm_grid_build")
        self._grid_info()

    def sensor(self):
        """kinetic sensor eps per cell (lbm_sensor), NaN for fine ghosts"""
        out = np.zeros(self.n)
        self._check(self._L.lbm_sensor(self.h, _ptr(out)), "lbm_sensor")
        return out

    def remesh(self, refine, solid=None):
        """adapt the grid to new refinement (and solid) masks, moving the
        state across (lbm_remesh); extent, levels and faces are kept"""
        ra, sa, keep = self._masks(refine, solid, self.n_levels)
        self._check(self._L.lbm_remesh(self.h, C.cast(ra, C.c_void_p),
                                       None if sa is None else C.cast(sa, C.c_void_p)), "lbm_remesh")
        self._grid_info()

    @staticmethod
    def _masks(refine, solid, n_levels):
        keep = []

        def mk(m):
            s = MaskC()
            if m is None:
                return s
            d = np.ascontiguousarray(m.data, dtype=np.uint8)
            keep.append(d)
            s.data = d.ctypes.data
            shape = tuple(reversed(d.shape))
            for a in range(3):
                s.lo[a] = int(m.lo[a]) if a < len(m.lo) else 0
                s.n[a] = int(shape[a]) if a < len(shape) else 1
            return s

        ra = (MaskC * max(1, n_levels - 1))(*[mk(r) for r in refine[: n_levels - 1]])
        sa = None
        if solid is not None and any(s is not None for s in solid):
            sa = (MaskC * n_levels)(*[mk(solid[l] if l < len(solid) else None) for l in range(n_levels)])
        return ra, sa, keep

    def _grid_info(self):
        n_levels, dim = self.n_levels, self.dim
        n = C.c_int64()
        npl = np.zeros(8, np.int64)
        ng = C.c_int64()
        eq = C.c_double()
        self._check(self._L.lbm_grid_info(self.h, C.byref(n), _ptr(npl), C.byref(ng), C.byref(eq)))
        self.n, self.n_per_level, self.n_ghosts, self.eq_fine = n.value, npl[:n_levels].copy(), ng.value, eq.value
        self.Q = LATTICE_Q[self.lattice]
        self.n_mom = 1 + dim + (1 if self.ddf else 0)

    def layout(self):
        """device placement: total slots, cells with explicit pull rows, and
        both per level"""
        ns, nx = C.c_int64(), C.c_int64()
        spl = np.zeros(8, np.int64)
        rpl = np.zeros(8, np.int64)
        self._check(self._L.lbm_layout_info(self.h, C.byref(ns), C.byref(nx), _ptr(spl), _ptr(rpl)),
                    "lbm_layout_info")
        return dict(slots=ns.value, exception_rows=nx.value, slots_per_level=spl[: self.n_levels].tolist(),
                    rows_per_level=rpl[: self.n_levels].tolist())

    def layout_export(self):
        """the brick layout's tables (slot of each cell, exception rows,
        neighbour bricks, exception masks, pull sources of the rows)"""
        info = self.layout()
        nb, nx = info["slots"] // 64, info["exception_rows"]
        nbp = 32 if self.dim == 3 else 16
        d = dict(slot_of=np.zeros(self.n, np.int32), xrow_of=np.zeros(self.n, np.int32),
                 nbrick=np.zeros((nb, nbp), np.int32), xmask=np.zeros(nb, np.uint64),
                 xnbr=np.zeros((self.Q - 1, nx), np.int32))
        self._check(self._L.lbm_layout_export(self.h, _ptr(d["slot_of"]), _ptr(d["xrow_of"]), _ptr(d["nbrick"]),
                                              _ptr(d["xmask"]), _ptr(d["xnbr"])), "lbm_layout_export")
        return d

    def export(self, parts=("coords", "level", "flags", "nbr", "child", "bc_src")):
        """canonical grid tables; `parts` selects which (the neighbour list of
        a large grid is big)"""
        n, Q = self.n, self.Q
        shapes = dict(coords=((n, 3), np.int32), level=((n,), np.int8), flags=((n,), np.uint8),
                      nbr=((n, Q - 1), np.int32), child=((self.n_ghosts, 1 << self.dim), np.int32),
                      bc_src=((n,), np.int32))
        d = {k: np.zeros(*shapes[k]) for k in parts}
        ptrs = [_ptr(d[k]) if k in d else None for k in ("coords", "level", "flags", "nbr", "child", "bc_src")]
        self._check(self._L.lbm_grid_export(self.h, *ptrs), "lbm_grid_export")
        return d

    def coords_levels(self):
        n = self.n
        coords, level = np.zeros((n, 3), np.int32), np.zeros(n, np.int8)
        self._check(self._L.lbm_grid_export(self.h, _ptr(coords), _ptr(level), None, None, None, None))
        return coords, level

    # ---- state -----------------------------------------------------------
    def init(self, moments):
        m = np.ascontiguousarray(moments, dtype=np.float64)
        assert m.shape == (self.n_mom, self.n), (m.shape, self.n_mom, self.n)
        self._check(self._L.lbm_init(self.h, _ptr(m)), "lbm_init")

    def init_workload(self, w):
        coords, level = self.coords_levels()
        self.init(w.initial_moments(coords, level))
        if getattr(w, "inflow_noise", None) is not None:
            self.set_inflow_noise(w.inflow_noise(coords, level))

    def step(self, n=1):
        self._check(self._L.lbm_step(self.h, int(n)), "lbm_step")

    def set_face(self, k, face):
        f = face_struct(face)
        self._check(self._L.lbm_set_face_bc(self.h, k, C.byref(f)), "lbm_set_face_bc")

    def graphs(self, on=True):
        """replay pairs of coarse steps from a HIP graph"""
        self._check(self._L.lbm_set_graphs(self.h, int(on)), "lbm_set_graphs")

    def set_inflow_noise(self, du):
        """du [3][n] (canonical order) added to the moving-wall velocity seen
        by each cell; None removes it"""
        if du is None:
            self._check(self._L.lbm_set_inflow_noise(self.h, None), "lbm_set_inflow_noise")
            return
        d = np.ascontiguousarray(du, dtype=np.float64)
        assert d.shape == (3, self.n)
        self._check(self._L.lbm_set_inflow_noise(self.h, _ptr(d)), "lbm_set_inflow_noise")

    def device_build(self, on=True):
        """build the tree and its layout on the GPU (default) or on the host"""
        self._check(self._L.lbm_set_device_build(self.h, int(on)), "lbm_set_device_build")

    def level_fusion(self, on=True):
        """one collide launch for all levels active at a substep"""
        self._check(self._L.lbm_set_level_fusion(self.h, int(on)), "lbm_set_level_fusion")

    def moments(self):
        out = np.zeros((self.n_mom, self.n))
        self._check(self._L.lbm_moments(self.h, _ptr(out)), "lbm_moments")
        return out

    def moments_device(self, out_tensor):
        """enqueue the moments into a CUDA tensor of n_mom * n float64; the
        caller's current stream waits for them"""
        import torch
        assert out_tensor.numel() >= self.n_mom * self.n
        out_tensor.record_stream(self.torch_stream)
        self.torch_stream.wait_stream(torch.cuda.current_stream(out_tensor.device))
        self._check(self._L.lbm_moments_device(self.h, C.c_void_p(out_tensor.data_ptr())),
                    "lbm_moments_device")
        torch.cuda.current_stream(out_tensor.device).wait_stream(self.torch_stream)

    def stats(self):
        s = Stats()
        self._check(self._L.lbm_stats_get(self.h, C.byref(s)), "lbm_stats_get")
        return dict(mass=s.mass, momentum=list(s.momentum)[: self.dim], energy=s.energy,
                    kinetic_energy=s.kinetic_energy,
                    updates=list(s.updates)[: self.n_levels], newton_calls=s.newton_calls,
                    newton_iterations=s.newton_iterations, newton_failures=s.newton_failures,
                    mlp_fallbacks=s.mlp_fallbacks, nonfinite_cells=s.nonfinite_cells,
                    coarse_steps=s.coarse_steps, newton_hist=list(s.newton_hist))

    def sums_device(self, out_ptr):
        """conserved sums into the device buffer at out_ptr (6 doubles:
        mass, momentum x/y/z, total energy, kinetic energy); enqueued only,
        allocation-free"""
        self._check(self._L.lbm_sums_device(self.h, C.c_void_p(int(out_ptr))), "lbm_sums_device")

    def sync(self):
        self._check(self._L.lbm_sync(self.h), "lbm_sync")

    def profile(self, on=True):
        self._check(self._L.lbm_profile_enable(self.h, int(on)), "lbm_profile_enable")

    def profile_read(self, level):
        n, ms, b = C.c_int64(), C.c_double(), C.c_double()
        self._check(self._L.lbm_profile_read(self.h, level, C.byref(n), C.byref(ms), C.byref(b)),
                    "lbm_profile_read")
        return n.value, ms.value, b.value

    def get_state(self):
        f = np.zeros((self.Q, self.n))
        g = np.zeros((self.Q, self.n)) if self.ddf else None
        lam = np.zeros((8, self.n))
        self._check(self._L.lbm_get_state(self.h, _ptr(f), _ptr(g), _ptr(lam)), "lbm_get_state")
        return f, g, lam

    def get_cells(self, cells):
        """state (f, g, lambda) of the listed canonical cells, [Q][n] each"""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        n = cells.size
        f = np.zeros((self.Q, n))
        g = np.zeros((self.Q, n)) if self.ddf else None
        lam = np.zeros((8, n))
        self._check(self._L.lbm_get_cells(self.h, _ptr(cells), n, _ptr(f), _ptr(g) if g is not None else None,
                                          _ptr(lam)), "lbm_get_cells")
        return f, g, lam

    def set_state(self, f, g=None, lam=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
        self._check(self._L.lbm_set_state(self.h, _ptr(f), _ptr(g), _ptr(lam)), "lbm_set_state")

    # ---- multiplier surrogate (D2Q21) ------------------------------------
    def mlp_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self._L.lbm_mlp_set_weights(self.h, _ptr(w), w.size), "lbm_mlp_set_weights")

    def mlp_get_weights(self):
        w = np.zeros(MLP_PARAMS, np.float32)
        self._check(self._L.lbm_mlp_get_weights(self.h, _ptr(w), w.size), "lbm_mlp_get_weights")
        return w

    def mlp_label(self, x):
        """Newton (cold start) multipliers of states x [n, 4] = (rho, ux, uy, T)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = x.shape[0]
        lam = np.zeros((n, 8))
        ok = np.zeros(n, np.uint8)
        it = np.zeros(n, np.int32)
        self._check(self._L.lbm_mlp_label(self.h, _ptr(x), n, _ptr(lam), _ptr(ok), _ptr(it)), "lbm_mlp_label")
        return lam, ok.astype(bool), it

    def mlp_predict(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        lam = np.zeros((x.shape[0], 8))
        self._check(self._L.lbm_mlp_predict(self.h, _ptr(x), x.shape[0], _ptr(lam)), "lbm_mlp_predict")
        return lam

    def mlp_grad(self, xh, th):
        xh = np.ascontiguousarray(xh, dtype=np.float32)
        th = np.ascontiguousarray(th, dtype=np.float32)
        g = np.zeros(MLP_PARAMS - 16, np.float32)
        loss = C.c_double()
        self._check(self._L.lbm_mlp_grad(self.h, _ptr(xh), _ptr(th), xh.shape[0], C.byref(loss), _ptr(g)),
                    "lbm_mlp_grad")
        return loss.value, g

    def mlp_train(self, x, lam, epochs=20, batch=1024, lr=2e-3, seed=5):
        x = np.ascontiguousarray(x, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        hist = np.zeros(epochs)
        self._check(self._L.lbm_mlp_train(self.h, _ptr(x), _ptr(lam), x.shape[0], epochs, batch, lr, seed,
                                          _ptr(hist)), "lbm_mlp_train")
        return hist
