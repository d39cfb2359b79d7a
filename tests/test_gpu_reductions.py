"""GPU parity of the global reductions (Sec. 4.1's reductions at the
coarse-step synchronisation point): mass, momentum, total energy (DDF) and
kinetic energy (the monitor of Sec. 5.2's convergence test) from the
library's FP64 block partials against the oracle's sums of the same state,
FP64 storage, on refined grids in 2-D and 3-D with walls, inflow and
outflow; and the Newton step histogram (Sec. 4.4) against the solve and
step counters."""
import numpy as np
import pytest

from gpu_util import run_pair, say
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "shear3": (lambda: W.shear(n=32, levels=3, kind="random", u0=0.03, nu_finest=0.02,
                               band=[(0.25, 0.75), (0.375, 0.625)]), 20),
    "cylinder/16": (lambda: W.cylinder(scale=16, steps=10), 10),
    "sphere/8": (lambda: W.sphere(scale=8, steps=3), 3),
    "airfoil/16": (lambda: W.airfoil(scale=16, steps=6), 6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sums_match_oracle(name):
    make, steps = CASES[name]
    w = make()
    say(f"[sums] {name}: {steps} coarse steps")
    mg, mo, level, s, o = run_pair(w, steps, "fp64")
    st = s.stats()
    ref = o.sums()
    D = w.dim
    ok = ~np.isnan(mo[0])
    vol = 0.5 ** (D * level[ok].astype(np.float64))
    umax = max(float(np.max(np.sqrt(sum(mo[1 + d][ok] ** 2 for d in range(D))))), 1e-3)
    mass = ref[0]
    ke = o.kinetic_energy()
    say(f"[sums] {name}: library mass {st['mass']!r} momentum {st['momentum']!r} energy {st['energy']!r} "
        f"KE {st['kinetic_energy']!r}")
    say(f"[sums] {name}: oracle  mass {ref[0]!r} momentum {list(ref[1:1 + D])!r} energy {ref[1 + D]!r} KE {ke!r}")
    assert abs(st["mass"] - mass) <= 1e-12 * abs(mass)
    for d in range(D):
        assert abs(st["momentum"][d] - ref[1 + d]) <= 1e-12 * abs(mass) * umax, (d, st["momentum"], ref)
    if w.collision.startswith("DDF"):
        assert abs(st["energy"] - ref[1 + D]) <= 1e-12 * abs(ref[1 + D])
    assert ke > 0
    assert abs(st["kinetic_energy"] - ke) <= 1e-12 * ke, (st["kinetic_energy"], ke)
    # the kinetic energy of the moments the library returns, summed here
    ke_m = 0.5 * np.sum(vol * mg[0][ok] * sum(mg[1 + d][ok] ** 2 for d in range(D)))
    assert abs(ke_m - ke) <= 1e-12 * ke
    if w.collision == "DDF_NEWTON":
        h = st["newton_hist"]
        assert sum(h) == st["newton_calls"] and st["newton_calls"] > 0
        assert sum(k * h[k] for k in range(15)) <= st["newton_iterations"]
        assert h[15] == 0 and st["newton_failures"] == 0
        say(f"[sums] {name}: Newton steps histogram {h[:8]}")
    else:
        assert sum(st["newton_hist"]) == 0
    s.close()
