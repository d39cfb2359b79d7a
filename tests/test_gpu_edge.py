"""GPU parity on the edge-case grids (partly filled bricks, wide stencils on
ragged extents, a grid smaller than one brick that wraps everywhere, an
empty refined level): FP64 storage against the oracle to relative L2 1e-12,
the Newton lattice (D2Q21) included."""
import numpy as np
import pytest

from edge_cases import edge_cases
from gpu_util import assert_within, compare, run_pair, say

pytestmark = pytest.mark.gpu

STEPS = {"ragged2d": 30, "ragged3d": 10, "ragged_d2q37": 20, "ragged_d2q21": 10, "tiny": 50, "empty_level": 20}


@pytest.mark.parametrize("name,w", edge_cases(), ids=[c[0] for c in edge_cases()])
def test_edge_grid_fp64_parity(name, w):
    steps = STEPS[name]
    say(f"[edge] {name}: {w.lattice} {w.collision} ext {w.ext}, {w.n_levels} levels, {steps} coarse steps")
    storage = "fp64"
    mg, mo, level, s, o = run_pair(w, steps, storage)
    err = compare(mg, mo, level, w.dim)
    say(f"[edge] {name}: {s.n} cells {list(s.n_per_level)}: {err}")
    assert_within(err, 1e-12)
    st = s.stats()
    counts = [int(n) for n in s.n_per_level]
    assert st["updates"] == [steps * (1 << l) * counts[l] for l in range(w.n_levels)]
    s.close()
