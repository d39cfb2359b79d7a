"""Refinement masks from the kinetic sensor (the adaptive runs of Sec. 8).

The finest level follows the cells whose sensor exceeds a threshold (0.2 in
the paper); every coarser level is the next finer one coarsened and grown
by a fixed number of its own cells, so the patches nest with a margin.
Fixed patches (e.g. around a body) are merged in.  Host-side integer work on
the grid's coordinates; the sensor itself comes from the device
(`LBM.sensor`, the C-ABI's lbm_sensor).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from .workloads import Mask


def _grow(m: np.ndarray, r: int, periodic: Sequence[bool]) -> np.ndarray:
    """dilate a dense mask by r cells along every axis (Chebyshev ball),
    wrapping across periodic axes and clipped at the others' edges;
    periodic[d] refers to coordinate axis d (array axis ndim-1-d)"""
    out = m.copy()
    nd = m.ndim
    for axis in range(nd):
        acc = out.copy()
        wrap = periodic[nd - 1 - axis]
        for k in range(1, r + 1):
            if wrap:
                acc |= np.roll(out, k, axis=axis) | np.roll(out, -k, axis=axis)
                continue
            acc[tuple(slice(k, None) if a == axis else slice(None) for a in range(nd))] |= \
                out[tuple(slice(None, -k) if a == axis else slice(None) for a in range(nd))]
            acc[tuple(slice(None, -k) if a == axis else slice(None) for a in range(nd))] |= \
                out[tuple(slice(k, None) if a == axis else slice(None) for a in range(nd))]
        out = acc
    return out


def _coarsen(m: np.ndarray) -> np.ndarray:
    """a cell of the coarser level is marked when any of its children is"""
    d = m.ndim
    shape = tuple((s + 1) // 2 for s in m.shape)
    out = np.zeros(shape, bool)
    for off in np.ndindex(*(2,) * d):
        sub = m[tuple(slice(o, None, 2) for o in off)]
        out[tuple(slice(0, s) for s in sub.shape)] |= sub
    return out


def sensor_masks(eps: np.ndarray, coords: np.ndarray, level: np.ndarray, ext: Sequence[int], n_levels: int,
                 threshold: float = 0.2, grow: int = 4,
                 fixed: Optional[List[Optional[Mask]]] = None,
                 periodic: Optional[Sequence[bool]] = None) -> List[Mask]:
    """Refinement masks (one per level below the finest) for the next grid.

    eps, coords, level: the current grid's sensor values, coordinates and
    levels (canonical order; NaN sensors are ignored).  The cells to refine
    into the finest level are those of level n_levels-2 over a flagged cell,
    grown by `grow` cells; each coarser mask is the finer one coarsened and
    grown by `grow` of its own cells (more than the lattice reach, so that
    successive interfaces stay apart).  Growth wraps across the `periodic`
    axes.  `fixed` masks are merged level by level."""
    dim = len(ext)
    per = list(periodic) if periodic is not None else [False] * dim
    top = n_levels - 2
    if top < 0:
        return []
    E = [tuple(int(e) << l for e in ext) for l in range(n_levels)]
    flagged = np.nan_to_num(eps, nan=-1.0) > threshold
    m = np.zeros(tuple(reversed(E[top])), bool)
    for lv in np.unique(level[flagged]):
        sel = flagged & (level == lv)
        x = coords[sel, :dim].astype(np.int64)
        if lv > top:
            x = x >> (int(lv) - top)
            m[tuple(x[:, a] for a in reversed(range(dim)))] = True
        else:
            s = 1 << (top - int(lv))
            for off in np.ndindex(*(s,) * dim):
                y = x * s + np.array(off)
                m[tuple(y[:, a] for a in reversed(range(dim)))] = True
    masks = [None] * (top + 1)
    masks[top] = _grow(m, grow, per)
    for l in range(top - 1, -1, -1):
        masks[l] = _grow(_coarsen(masks[l + 1]), grow, per)
    out = []
    for l in range(top + 1):
        d = masks[l]
        if fixed is not None and l < len(fixed) and fixed[l] is not None:
            d = d | fixed[l].dense(E[l]).astype(bool)
        if l > 0:
            # a finer patch must lie inside the coarser one
            d &= np.kron(out[l - 1].data.astype(bool), np.ones((2,) * dim, bool))[
                tuple(slice(0, s) for s in d.shape)]
        out.append(Mask(d.astype(np.uint8), (0,) * dim))
    return out
