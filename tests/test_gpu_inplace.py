"""In-place (AA-pattern) streaming on one population buffer against the
two-buffer path: the same arithmetic on the same values, so moments,
populations, conserved sums and the sensor must be bit-identical after odd
and even step counts, launched and replayed from a HIP graph; the
two-buffer path is itself tied to the oracle by the parity tests, and one
case here checks the oracle directly."""
import numpy as np
import pytest

from gpu_util import compare, say
from oracle.oracle import Oracle
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu


def one_level(lattice, collision, n, kind="random", T0=1.0):
    w = W.shear(n=n, levels=1, lattice=lattice, collision=collision, kind=kind, u0=0.03, nu_finest=0.02, T0=T0)
    return w


def cavity(lattice, collision):
    return W.cavity(n=48, levels=1, lattice=lattice, collision=collision)


def refined(lattice, collision, n, levels, T0=1.0):
    w = W.shear(n=n, levels=levels, lattice=lattice, collision=collision, kind="random", u0=0.03, nu_finest=0.02,
                T0=T0)
    return w


CASES = [("shear D2Q9 RR", lambda: one_level("D2Q9", "RR", 32), "fp32"),
         ("shear D2Q9 BGK", lambda: one_level("D2Q9", "BGK", 32), "fp64"),
         ("shear D3Q27 RR", lambda: one_level("D3Q27", "RR", 12), "fp32"),
         ("shear D3Q27 RR fp16", lambda: one_level("D3Q27", "RR", 12), "fp16"),
         ("shear D2Q13 RR", lambda: one_level("D2Q13", "RR", 32), "fp64"),
         ("shear D2Q37 DDF", lambda: one_level("D2Q37", "DDF_POLY", 32), "fp32"),
         ("shear D2Q21 Newton", lambda: one_level("D2Q21", "DDF_NEWTON", 32, T0=0.65), "fp64"),
         ("cavity D2Q9 BGK", lambda: cavity("D2Q9", "BGK"), "fp64"),
         ("cavity D2Q21 RR", lambda: cavity("D2Q21", "RR"), "fp32"),
         # across refinement interfaces: coalescence, explosion and the
         # fine ghosts' own links read and written in each level's phase
         ("refined shear D2Q9 RR 3 levels", lambda: refined("D2Q9", "RR", 32, 3), "fp32"),
         ("refined shear D2Q9 BGK 3 levels", lambda: refined("D2Q9", "BGK", 32, 3), "fp64"),
         ("refined shear D3Q27 RR", lambda: refined("D3Q27", "RR", 12, 2), "fp32"),
         ("refined shear D3Q27 RR fp16", lambda: refined("D3Q27", "RR", 12, 2), "fp16"),
         ("refined shear D2Q13 RR", lambda: refined("D2Q13", "RR", 32, 3), "fp64"),
         ("refined shear D2Q37 DDF", lambda: refined("D2Q37", "DDF_POLY", 32, 2), "fp32"),
         ("refined shear D2Q21 Newton", lambda: refined("D2Q21", "DDF_NEWTON", 32, 2, T0=0.65), "fp64"),
         ("refined cavity D2Q9 BGK (the 64 x 64 cavity, walls and lid)", lambda: W.cavity(n=64, steps=1), "fp64"),
         ("refined cavity D2Q9 RR fp32", lambda: W.cavity(n=64, steps=1, collision="RR", storage="fp32"), "fp32"),
         # open faces: Neumann and equilibrium boundary layers filled in each
         # phase, sponge, moving-wall inflow
         ("cylinder 1/16 (Neumann, sponge, inflow)", lambda: W.cylinder(scale=16, steps=1), "fp32"),
         ("cylinder 1/16 fp64", lambda: W.cylinder(scale=16, steps=1, storage="fp64"), "fp64"),
         ("sphere 1/8 (Neumann, inflow)", lambda: W.sphere(scale=8, steps=1), "fp32"),
         # FP16 with a moving wall: in place the bounced-back population is
         # stored with its moving-wall term, so it is rounded to FP16 once
         # more than the two-buffer pull, which adds the term after loading;
         # compared within a tolerance (test_in_place_fp16_moving_wall)
         ("airfoil 1/16 (equilibrium faces, D2Q21 Newton)", lambda: W.airfoil(scale=16, steps=1), "fp64"),
         ("Sod 256 (D2Q37, Neumann)", lambda: W.sod(nx=256, ny=8), "fp32")]


def pair(w, storage):
    a = B.LBM.from_workload(w, storage=storage)
    b = B.LBM.from_workload(w, storage=storage, in_place=True)
    coords, level = a.coords_levels()
    m0 = w.initial_moments(coords, level)
    a.init(m0)
    b.init(m0)
    return a, b


def test_in_place_fp16_moving_wall():
    """the FP16 sphere (moving-wall inflow) in place against two buffers:
    the only difference is the extra FP16 rounding of the bounced-back
    populations next to the inflow, far below the FP16 storage error"""
    w = W.sphere(scale=8, steps=1)
    a, b = pair(w, "fp16")
    for n in (1, 2, 5):
        a.step(n)
        b.step(n)
        ma, mb = a.moments(), b.moments()
        ok = np.isfinite(ma) & np.isfinite(mb)
        assert np.array_equal(np.isfinite(ma), np.isfinite(mb))
        d = float(np.max(np.abs(ma[ok] - mb[ok])))
        say(f"[in-place] sphere 1/8 fp16: max |moment difference| after {n} more steps {d:.2e}")
        assert d < 1e-4, d
    a.close()
    b.close()


@pytest.mark.parametrize("name,make,storage", CASES, ids=[c[0] for c in CASES])
def test_in_place_equals_two_buffers(name, make, storage):
    w = make()
    a, b = pair(w, storage)
    for n in (1, 2, 5):  # odd and even totals (1, 3, 8)
        a.step(n)
        b.step(n)
        ma, mb = a.moments(), b.moments()
        assert np.array_equal(ma, mb, equal_nan=True), (name, n, np.nanmax(np.abs(ma - mb)))
        fa, ga, la = a.get_state()
        fb, gb, lb = b.get_state()
        assert np.array_equal(fa, fb) and (ga is None or np.array_equal(ga, gb))
        assert np.array_equal(a.sensor(), b.sensor(), equal_nan=True)
    say(f"[in-place] {name} {storage}: identical after 1, 3 and 8 steps")
    a.close()
    b.close()


def test_in_place_graph_replay_and_oracle():
    """graph replay from both parities of the in-place state, and the
    oracle, on the two-level-free cavity with a moving lid (walls push back
    with the moving-wall correction)"""
    w = cavity("D2Q9", "RR")
    a, b = pair(w, "fp64")
    o = Oracle.from_workload(w)
    e = o.export()
    o.init(w.initial_moments(e["coords"], e["level"]))
    b.graphs(True)
    for n in (3, 4, 7):
        a.step(n)
        b.step(n)
        o.step(n)
        assert np.array_equal(a.moments(), b.moments(), equal_nan=True)
    err = compare(b.moments(), o.moments(), e["level"], 2)
    say(f"[in-place] cavity D2Q9 RR fp64 vs oracle after 14 steps: {err}")
    assert err["u"] <= 1e-12 and err["rho"] <= 1e-12, err
    a.close()
    b.close()


def test_in_place_refined_graph_replay_and_oracle():
    """the two-level 64 x 64 cavity (walls, moving lid, an interface meeting
    both side walls) streamed in place and replayed from HIP graphs: equal
    to two buffers bit for bit, and to the oracle at the FP64 bar"""
    w = W.cavity(n=64, steps=1)
    a, b = pair(w, "fp64")
    o = Oracle.from_workload(w)
    e = o.export()
    o.init(w.initial_moments(e["coords"], e["level"]))
    b.graphs(True)
    for n in (3, 4, 7):
        a.step(n)
        b.step(n)
        o.step(n)
        assert np.array_equal(a.moments(), b.moments(), equal_nan=True)
    err = compare(b.moments(), o.moments(), e["level"], 2)
    say(f"[in-place] refined cavity D2Q9 BGK fp64 vs oracle after 14 steps: {err}")
    assert err["u"] <= 1e-12 and err["rho"] <= 1e-12, err
    a.close()
    b.close()
