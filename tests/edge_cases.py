"""Small grids at the edges of what the brick layout handles, shared by the
host and GPU tests:
- extents that are no multiple of the 64-cell bricks (partly filled bricks,
  holes), 2-D and 3-D, with a refined box in the interior;
- the same for the wide-stencil D2Q37 and D2Q21 lattices (reach 3);
- one level smaller than a single brick, periodic in both directions, so
  that every pull source wraps;
- a second level declared but left empty by its refinement mask."""
import numpy as np

from paper_2504_04465_amd import workloads as W


def _box_grid(ext, lattice, collision, box, levels=2):
    w = W.shear(n=max(ext), levels=1, lattice=lattice, collision=collision, nu_finest=0.05,
                kind="random", u0=0.03)
    w.ext = tuple(ext)
    w.n_levels = levels
    w.refine = [W._box_mask(w.ext, len(ext), 0, *box)] if levels > 1 else []
    w.solid = [None] * levels
    return w


def edge_cases():
    return [
        ("ragged2d", _box_grid((21, 13), "D2Q9", "RR", ((6, 4), (15, 9)))),
        ("ragged3d", _box_grid((11, 9, 7), "D3Q27", "RR", ((3, 2, 2), (8, 7, 5)))),
        ("ragged_d2q37", _box_grid((37, 29), "D2Q37", "DDF_POLY", ((10, 9), (27, 20)))),
        ("ragged_d2q21", _box_grid((37, 29), "D2Q21", "DDF_NEWTON", ((10, 9), (27, 20)))),
        ("tiny", _box_grid((3, 5), "D2Q9", "BGK", None, levels=1)),
        ("empty_level", _box_grid((16, 16), "D2Q9", "RR", ((0, 0), (0, 0)))),
    ]
