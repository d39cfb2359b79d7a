"""Dependency cones of single cells for sampled parity checks on grids the
oracle cannot run whole: pick bulk cells whose cone (radius reach x
substeps) holds only bulk cells of their level, and advance a cone with the
oracle's single-cell collision and pull streaming (Sec. 4.5: level l takes
2^l substeps per coarse step)."""
import numpy as np


def level_lookup(coords, level, flags, l, dim):
    """dense index of the level-l cells over their bounding box; cells that
    are not plain bulk cells (any flag) are marked -2"""
    sel = np.nonzero(level == l)[0]
    xyz = coords[sel, :dim].astype(np.int64)
    lo = xyz.min(0)
    n = xyz.max(0) - lo + 1
    tab = np.full(tuple(n[::-1]), -1, np.int64)
    idx = tuple((xyz - lo)[:, d] for d in reversed(range(dim)))
    tab[idx] = np.where(flags[sel] == 0, sel, -2)
    return tab, lo


def find(tab, lo, pts):
    """cell index at level coordinates pts [m, dim], -1 outside"""
    q = pts - lo
    n = np.array(tab.shape[::-1])
    ok = np.all((q >= 0) & (q < n), axis=1)
    out = np.full(len(pts), -1, np.int64)
    out[ok] = tab[tuple(q[ok, d] for d in reversed(range(pts.shape[1])))]
    return out


def sample_cones(tab, lo, lat_c, reach, steps, rng, k, dim):
    """k bulk cells whose dependency cone (radius reach * steps) holds only
    bulk cells of the level; returns centres and cone offsets"""
    r = reach * steps
    ax = np.arange(-r, r + 1)
    offs = np.stack(np.meshgrid(*([ax] * dim), indexing="ij"), -1).reshape(-1, dim)
    cand = np.argwhere(tab[(slice(r, -r),) * dim] >= 0)[:, ::-1] + r + lo
    rng.shuffle(cand)
    out = []
    for p in cand:
        cells = find(tab, lo, p + offs)
        if np.all(cells >= 0):
            out.append(cells)
            if len(out) == k:
                break
    assert len(out) == k, f"only {len(out)} clean cones"
    return np.array(out), offs


def advance_cone(o, tau, offs, f, g, lam, lat_c, reach, steps, dim):
    """oracle: `steps` substeps of collide + pull-stream on one cone
    [n_off, Q] (g likewise); returns the centre's populations"""
    Q = f.shape[1]
    pos = {tuple(p): j for j, p in enumerate(offs)}
    alive = np.ones(len(offs), bool)
    for s in range(steps):
        fs, gs, ls = np.zeros_like(f), (None if g is None else np.zeros_like(g)), lam.copy()
        for j in np.nonzero(alive)[0]:
            a, b, lm, _ = o.collide(tau, f[j], None if g is None else g[j], lam[j])
            fs[j] = a
            if g is not None:
                gs[j] = b
            ls[j] = lm
        r_new = reach * (steps - s - 1)
        nf, ng = np.zeros_like(f), (None if g is None else np.zeros_like(g))
        new_alive = np.all(np.abs(offs) <= r_new, axis=1)
        for j in np.nonzero(new_alive)[0]:
            for i in range(Q):
                src = pos[tuple(offs[j] - lat_c[i, :dim])]
                nf[j, i] = fs[src, i]
                if g is not None:
                    ng[j, i] = gs[src, i]
        f, g, lam, alive = nf, ng, ls, new_alive
    centre = pos[(0,) * dim]
    return f[centre], (None if g is None else g[centre])
