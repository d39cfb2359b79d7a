"""Mesh adaptation of the oracle (Sec. 8, methodology of the adaptive runs).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the library.

After a new tree is built, every new cell takes its populations from the old
tree: copied where the old tree has a flow cell at the same place and level,
copied from the old cell that contains it where the old tree is coarser there
(uniform explosion), and averaged over the old cells inside it, weighted by
their volume, where the old tree is finer (coalescence).  The sources are the
old cells other than fine ghosts, taken at the synchronisation point (coarse
ghosts with their unknown populations coalesced): in the band where two
levels overlap the coarse ghost carries the state, and these cells tile the
fluid domain once.  Ghost cells of the new tree are filled by the same rule.
The multipliers of the numerical equilibrium move the same way.

Plain loops over cells and a dictionary of the old flow cells, FP64.
"""
import itertools

import numpy as np

from .oracle import F_FINE_GHOST


def sources(old, new, dim):
    """For every new cell, the list of (old cell, weight).  old / new are
    export dictionaries (coords [n][3], level [n], flags [n])."""
    flow = {}
    for c in range(len(old["level"])):
        if old["flags"][c] & F_FINE_GHOST:
            continue
        x = old["coords"][c]
        flow[(int(old["level"][c]), int(x[0]), int(x[1]), int(x[2]))] = c
    deepest = int(np.max(old["level"])) if len(old["level"]) else 0
    offsets = list(itertools.product((0, 1), repeat=dim))
    out = []
    for j in range(len(new["level"])):
        lev = int(new["level"][j])
        x = [int(v) for v in new["coords"][j]]
        found = None
        # the old flow cell at this place, at this level or coarser
        for up in range(lev, -1, -1):
            s = lev - up
            key = (up, x[0] >> s, x[1] >> s, x[2] >> s)
            if key in flow:
                found = [(flow[key], 1.0)]
                break
        if found is None:
            # the old flow cells inside, each weighted by its share of the volume
            acc = []

            def inside(level, cx, share):
                if level >= deepest:
                    return
                for o in offsets:
                    ch = [2 * cx[0] + o[0], 2 * cx[1] + (o[1] if dim > 1 else 0),
                          2 * cx[2] + (o[2] if dim > 2 else 0)]
                    if dim < 3:
                        ch[2] = 0
                    key = (level + 1, ch[0], ch[1], ch[2])
                    w = share / len(offsets)
                    if key in flow:
                        acc.append((flow[key], w))
                    else:
                        inside(level + 1, ch, w)

            inside(lev, x, 1.0)
            total = sum(w for _, w in acc)
            if not acc or total <= 0.0:
                raise ValueError(f"new cell {j} (level {lev}, {x}) covers no old flow cell")
            found = [(c, w / total) for c, w in acc]
        out.append(found)
    return out


def transfer(src, arrays):
    """arrays: per-cell state of the old tree, [n_old][k] each; returns the
    new tree's [n_new][k] arrays, sum of weight x old value per new cell."""
    outs = []
    for a in arrays:
        if a is None:
            outs.append(None)
            continue
        b = np.zeros((len(src), a.shape[1]))
        for j, lst in enumerate(src):
            v = np.zeros(a.shape[1])
            for c, w in lst:
                v = v + w * a[c]
            b[j] = v
        outs.append(b)
    return outs


def remesh(o, refine, solid=None):
    """Adapt the oracle `o` to new refinement masks (same extent, levels and
    faces) and move its state across."""
    old = o.export()
    f, g, lam = o.sync_state()
    o.grid(o.dim, o._ext, o.n_levels, refine, solid if solid is not None else [None] * o.n_levels, o._faces)
    new = o.export()
    src = sources(old, new, o.dim)
    f2, g2, lam2 = transfer(src, [f, g, lam])
    o.set_state(f2, g2, lam2)
    return src
