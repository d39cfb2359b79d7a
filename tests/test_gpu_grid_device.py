"""The grid and brick layout built on the GPU against the host builder (which
test_lib_host ties to the oracle's own grid builder bit for bit): every
canonical table and every layout table must be identical, integer for
integer, on the small parity grids, the ragged and degenerate edge cases,
and full-size workloads; invalid masks must fail with the same code and
text; a run and a remesh on the device-built grid must give the same bits
as on the host-built one."""
import time

import numpy as np
import pytest

from edge_cases import edge_cases
from gpu_util import say
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu


def build(w, device, storage=None):
    s = B.LBM(w.lattice, w.collision, storage or w.storage, nu_finest=w.nu_finest, T0=w.T0, gamma=w.gamma,
              sensor_A=w.sensor_A, sensor_on=w.sensor_on, trace_eq=w.trace_eq, newton_tol=w.newton_tol,
              newton_max_it=w.newton_max_it, warm_start=w.warm_start)
    s.device_build(device)
    t0 = time.perf_counter()
    s.grid(w.dim, w.ext, w.n_levels, w.refine, w.solid, w.faces)
    return s, time.perf_counter() - t0


def same_grid(a, b, name):
    assert a.n == b.n and list(a.n_per_level) == list(b.n_per_level), name
    ea, eb = a.export(), b.export()
    for k in ea:
        assert ea[k].shape == eb[k].shape and np.array_equal(ea[k], eb[k]), (name, k)
    assert a.layout() == b.layout(), name
    la, lb = a.layout_export(), b.layout_export()
    for k in la:
        assert la[k].shape == lb[k].shape and np.array_equal(la[k], lb[k]), (name, k)


def small_cases():
    out = [("cavity", W.cavity(n=16, steps=1)), ("cavity64", W.cavity(n=64, steps=1)),
           ("shear3", W.shear(n=16, levels=3, steps=1)), ("cyl", W.cylinder(scale=16, steps=1)),
           ("sod", W.sod(nx=128, ny=8, steps=1)), ("airfoil", W.airfoil(scale=16, steps=1)),
           ("sphere", W.sphere(scale=8, steps=1)),
           ("shear_q13", W.shear(n=32, levels=3, lattice="D2Q13", collision="DDF_NEWTON", T0=0.35))]
    return out + edge_cases()


@pytest.mark.parametrize("name,w", small_cases(), ids=[c[0] for c in small_cases()])
def test_device_grid_equals_host_grid(name, w):
    a, _ = build(w, True)
    b, _ = build(w, False)
    same_grid(a, b, name)
    a.close()
    b.close()


FULL = [("cylinder", lambda: W.cylinder(scale=1, steps=1)), ("sphere", lambda: W.sphere(scale=1, steps=1)),
        ("airfoil", lambda: W.airfoil(scale=1, steps=1)), ("vortex", lambda: W.vortex(n=2048, levels=3, steps=1)),
        ("sod", lambda: W.sod(steps=1))]


@pytest.mark.parametrize("name,make", FULL, ids=[c[0] for c in FULL])
def test_device_grid_full_size(name, make):
    """full-size grids (the sphere has 64.7 M cells): identical tables, and
    the build time of both paths"""
    w = make()
    a, ta = build(w, True)
    b, tb = build(w, False)
    same_grid(a, b, name)
    say(f"[grid build] {name}: {a.n} cells, device {ta * 1e3:.0f} ms, host {tb * 1e3:.0f} ms")
    a.close()
    b.close()


def test_device_grid_mask_errors_match():
    bad = [W.shear(n=16, levels=3, steps=1, band=[(0.5, 1.0), (0.5, 0.75)])]
    w = W.shear(n=16, levels=3, steps=1)
    w.refine[1] = W.Mask(np.ones((4, 32), np.uint8), (0, 0))
    bad.append(w)
    w = W.cavity(n=16, steps=1)
    w.faces[1] = W.Face("periodic")  # unpaired periodic face
    bad.append(w)
    w = W.shear(n=24, levels=2, steps=1)
    w.refine = [W.Mask(np.ones((2, 2), np.uint8), (40, 40))]  # window outside its level
    bad.append(w)
    for w in bad:
        msgs = []
        for device in (True, False):
            with pytest.raises(B.LbmError) as e:
                build(w, device)
            msgs.append((e.value.code, str(e.value).split(":", 2)[-1]))
        assert msgs[0] == msgs[1], msgs


def test_device_grid_run_and_remesh_bit_identical():
    """the cylinder stepped on both grids, and the vortex remeshed on both
    paths: the same moments bit for bit"""
    w = W.cylinder(scale=8, steps=4)
    a, _ = build(w, True, "fp64")
    b, _ = build(w, False, "fp64")
    for s in (a, b):
        s.init_workload(w)
        s.step(3)
    assert np.array_equal(a.moments(), b.moments(), equal_nan=True)
    a.close()
    b.close()
    w = W.vortex(n=256, levels=3, steps=8)
    a, _ = build(w, True, "fp64")
    b, _ = build(w, False, "fp64")
    for s in (a, b):
        s.init_workload(w)
        s.step(2)
    times = []
    for k in (1, 2):
        m = w.patch(k * w.ext[0] / 64 / 0.05)
        t = []
        for s in (a, b):
            t0 = time.perf_counter()
            s.remesh(m)
            s.sync()
            t.append(time.perf_counter() - t0)
            s.step(1)
        times.append(t)
        same_grid(a, b, f"vortex remesh {k}")
        assert np.array_equal(a.moments(), b.moments(), equal_nan=True)
    say(f"[remesh] vortex 256: device {times[-1][0] * 1e3:.1f} ms, host {times[-1][1] * 1e3:.1f} ms")
    a.close()
    b.close()
