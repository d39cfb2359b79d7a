"""Concurrent levels (lbm_set_level_fusion): the collides of every level
active at a substep in one launch give the same state, bit for bit, as one
launch per level, on grids with two to four levels in 2-D and 3-D (walls,
moving walls, Neumann faces with the sponge, the refined band of the shock
tube), launched and replayed from HIP graphs, with eager steps and
read-backs between the replays."""
import numpy as np
import pytest

from gpu_util import say
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "cavity": lambda: W.cavity(n=32, steps=1),
    "cylinder/8": lambda: W.cylinder(scale=8, steps=1),
    "sphere/8": lambda: W.sphere(scale=8, steps=1),
    "sod256": lambda: W.sod(nx=256, ny=8, steps=1),
    "shear3-d2q13-rr": lambda: W.shear(n=32, levels=3, lattice="D2Q13", collision="RR", kind="random", u0=0.03,
                                       nu_finest=0.02, band=[(0.25, 0.75), (0.375, 0.625)]),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("graphs", [False, True])
def test_fused_levels_bit_identical(name, graphs):
    w = CASES[name]()
    a = B.LBM.from_workload(w, storage="fp32")
    b = B.LBM.from_workload(w, storage="fp32")
    a.level_fusion(False)
    for s in (a, b):
        s.init_workload(w)
        s.step(1)  # the first step after initialisation reads pre-collision input
        if graphs:
            s.graphs(True)
    for rep in range(3):
        a.step(2)
        b.step(2)
        fa, ga, _ = a.get_state()
        fb, gb, _ = b.get_state()
        assert np.array_equal(fa, fb), (name, rep)
        if ga is not None:
            assert np.array_equal(ga, gb), (name, rep)
        a.step(1)
        b.step(1)
        a.sync()
        b.sync()
    sa, sb = a.stats(), b.stats()
    assert sa["updates"] == sb["updates"] and sa["mass"] == sb["mass"]
    say(f"[fusion] {name} graphs={graphs}: {sb['coarse_steps']} coarse steps identical to per-level launches")
    a.close()
    b.close()
