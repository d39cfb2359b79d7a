"""The cone machinery of the full-size sampled parity tests, checked against
the oracle itself: advancing a bulk cell's cone with single-cell collisions
and pull streaming reproduces the oracle's own coarse step on a small
refined grid (every level, 1 to 4 substeps)."""
import numpy as np
import pytest

from cones import advance_cone, level_lookup, sample_cones
from oracle.oracle import Oracle
from paper_2504_04465_amd import workloads as W


@pytest.mark.parametrize("name,w,levels", [
    ("sphere", W.sphere(scale=8, steps=1), [0, 2]),
    ("cylinder", W.cylinder(scale=4, steps=1), [0, 1, 2, 3]),
    ("airfoil", W.airfoil(scale=8, steps=1), [0, 2]),
])
def test_cone_advance_matches_oracle_step(name, w, levels):
    o = Oracle.from_workload(w)
    o.init_workload(w)
    o.step(2)
    e = o.export()
    coords, level, flags = e["coords"], e["level"].astype(np.int64), e["flags"]
    f0, g0, l0 = o.state()
    o.step(1)
    f1, g1, _ = o.state()
    reach = int(np.max(np.abs(o.c)))
    rng = np.random.default_rng(1)
    for l in levels:
        tab, lo = level_lookup(coords, level, flags, l, w.dim)
        cc, offs = sample_cones(tab, lo, o.c, reach, 1 << l, rng, 3, w.dim)
        for m in range(len(cc)):
            j = cc[m]
            rf, rg = advance_cone(o, o.tau(l), offs, f0[j].copy(), None if g0 is None else g0[j].copy(),
                                  l0[j].copy(), o.c, reach, 1 << l, w.dim)
            c = cc[m][len(offs) // 2]
            assert np.max(np.abs(rf - f1[c])) <= 1e-13 * np.max(np.abs(f1[c])), (name, l, m)
            if g0 is not None:
                assert np.max(np.abs(rg - g1[c])) <= 1e-13 * np.max(np.abs(g1[c])), (name, l, m)
