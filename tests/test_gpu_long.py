"""FP64 parity over long runs: 1000 coarse steps on the scaled cylinder
(four levels, D2Q9 RR, Ladd inflow, Neumann faces with the sponge), the
scaled sphere (three octree levels, D3Q27 RR) and the scaled airfoil (three
levels, D2Q21 Newton equilibrium with the Mach ramp and the kinetic
sensor), and the D2Q37 shock tube at its full benchmark size (4096 x 8
coarse cells with the refined band, to the end time), all against the FP64
oracle from the same seeded start: relative L2 <= 1e-12 of density and
velocity, the worst cell within 10x that.  The shock tube's FP32 storage is
held to the sensor-switching bound of its small twin, and both precisions
to the exact Riemann solution.  Both sides advance in chunks of coarse
steps, with progress printed after each chunk."""
import math
import sys

import numpy as np
import pytest

import riemann_exact
from gpu_util import assert_within, compare, say
from oracle.oracle import Oracle
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu


def run_long(name, w, steps, storage, chunk=100):
    o = Oracle.from_workload(w)
    s = B.LBM.from_workload(w, storage=storage)
    coords, level = s.coords_levels()
    assert np.array_equal(coords, o.export()["coords"])
    m0 = w.initial_moments(coords, level)
    o.init(m0)
    s.init(m0)
    if w.inflow_noise is not None:
        du = w.inflow_noise(coords, level)
        o.set_inflow_noise(du)
        s.set_inflow_noise(du)
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        if w.schedule is None:
            o.step(n)
            s.step(n)
        else:
            for k in range(done, done + n):
                for face, f in w.schedule(k).items():
                    o.set_face(face, f)
                    s.set_face(face, f)
                o.step(1)
                s.step(1)
        done += n
        say(f"[long] {name} {storage}: {done}/{steps} coarse steps")
    return s.moments(), o.moments(), level, s, o


def alpha_band(eps, A_band):
    """index of the sensor's relaxation band (Eq. shock_function)"""
    return np.where(eps < 0.01, 0, np.where(eps < 0.1, 1, np.where(eps < 1.0, 2, 3)))


LONG = {
    # the 1/8 twin at the full-size relaxation times (Re / 8): at Re 150 the
    # scaled coarse level sits at tau = 0.512 and its wake blows up at the
    # outflow after ~800 coarse steps, in the oracle as on the GPU
    "cylinder/8": lambda: W.cylinder(scale=8, steps=1000, Re=150.0 / 8),
    "sphere/8": lambda: W.sphere(scale=8, steps=1000),
    "airfoil/16": lambda: W.airfoil(scale=16, steps=1000),
}


@pytest.mark.parametrize("name", list(LONG))
def test_fp64_1000_coarse_steps(name):
    w = LONG[name]()
    mg, mo, level, s, o = run_long(name, w, 1000, "fp64")
    err = compare(mg, mo, level, w.dim)
    say(f"[long] {name} fp64 after 1000 coarse steps: {err}")
    if w.sensor_on:
        # the sensor's relaxation band of every cell at the end, both sides
        eg, eo = s.sensor(), o.sensor()
        ok = ~np.isnan(eo)
        flips = int(np.sum(alpha_band(eg[ok], w.sensor_A) != alpha_band(eo[ok], w.sensor_A)))
        say(f"[long] {name}: sensor bands differing at the end: {flips} of {int(ok.sum())} cells")
        assert flips == 0
    assert_within(err, 1e-12)
    st = s.stats()
    if w.collision == "DDF_NEWTON":
        assert st["newton_failures"] == 0
    s.close()


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_sod_full_size(storage):
    """D2Q37 DDF shock tube at the benchmark size: 4096 x 8 coarse cells,
    refined band [1024, 3072), kinetic sensor, to the end time (1016 coarse
    steps).  Over this many steps the run is chaotic: the sensor's
    piecewise-constant relaxation (Eq. shock_function) flips a cell's band
    on a rounding-level change, and the oracle started from a density
    perturbed by 1e-15 (relative) ends 4e-3 (relative L2) away from itself
    (at 1024 x 8 and 254 steps the same perturbation grows only to 1e-10;
    without the sensor the inviscid tube blows up).  Parity is therefore:
    the library is no further from the oracle than the oracle is from its
    own perturbed run (within 3x), and both meet the exact Riemann solution
    equally well.  The 256 x 8 twin is held to 1e-12 in
    test_gpu_parity.py."""
    w = W.sod(nx=4096, ny=8)
    mg, mo, level, s, o = run_long("sod4096", w, w.steps, storage, chunk=200)
    err = compare(mg, mo, level, w.dim)
    say(f"[long] sod4096 {storage}: {err}")
    p = Oracle.from_workload(w)
    e = p.export()
    m0 = w.initial_moments(e["coords"], e["level"])
    m0[0] *= 1.0 + 1e-15 * np.random.default_rng(0).standard_normal(m0.shape[1])
    p.init(m0)
    for k in range(0, w.steps, 200):
        p.step(min(200, w.steps - k))
        say(f"[long] sod4096 perturbed oracle: {min(k + 200, w.steps)}/{w.steps} coarse steps")
    self_err = compare(p.moments(), mo, level, w.dim)
    say(f"[long] sod4096 oracle vs its 1e-15-perturbed run: {self_err}")
    for q in ("rho", "u", "T"):
        assert err[q] <= 3.0 * self_err[q], (q, err, self_err)
    # L1 of the density against the exact Riemann solution, both sides
    e = o.export()
    ok = ~np.isnan(mo[0])
    lev = e["level"][ok]
    xc = (e["coords"][ok, 0] + 0.5) / 2.0 ** lev
    t = w.steps * math.sqrt(w.T0)
    ex = riemann_exact.sample((xc - 4096 / 2) / t, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    vol = 0.25 ** lev
    l1_o = float(np.sum(vol * np.abs(mo[0][ok] - ex[0])) / np.sum(vol))
    l1_g = float(np.sum(vol * np.abs(mg[0][ok] - ex[0])) / np.sum(vol))
    say(f"[long] sod4096 {storage}: L1(rho - exact) oracle {l1_o:.3e}, library {l1_g:.3e}")
    # the oracle measures 2.0e-3 here (discontinuities converge at first
    # order); the chaotic differences leave the error against the exact
    # solution unchanged to a few per cent
    assert l1_o < 3e-3 and abs(l1_g - l1_o) <= 0.05 * l1_o
    s.close()
