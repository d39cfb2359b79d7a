"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: the oracle cannot run these grids, so a sample of bulk cells (away
from interfaces, boundary layers and bodies) is checked one by one.  The
library's state of each sampled cell's dependency cone is read before a
coarse step (lbm_get_cells); the oracle advances that cone with its own
single-cell collision and pull streaming for the 2^l substeps of level l
(Sec. 4.5), and the result must match the library's state after the step.
The sampled populations are compared in the storage precision: relative
error of the sample, max |f_gpu - f_oracle| / max |f_oracle|."""
import numpy as np
import pytest

from cones import advance_cone, level_lookup, sample_cones
from gpu_util import say
from oracle.oracle import Oracle
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu


def sampled_check(w, storage, levels, k, tol, steps_before=3, seed=0):
    s = B.LBM.from_workload(w, storage=storage)
    s.init_workload(w)
    for st in range(steps_before):
        if w.schedule is not None:
            for face, fv in w.schedule(st).items():
                s.set_face(face, fv)
        s.step(1)
    e = s.export(parts=("coords", "level", "flags"))
    coords, level, flags = e["coords"], e["level"].astype(np.int64), e["flags"]
    del e
    o = Oracle.from_workload(small_twin(w), nu_finest=w.nu_finest)
    lat_c = o.c
    reach = int(np.max(np.abs(lat_c)))
    rng = np.random.default_rng(seed)
    cones = {}
    for l in levels:
        tab, lo = level_lookup(coords, level, flags, l, w.dim)
        cones[l] = sample_cones(tab, lo, lat_c, reach, 1 << l, rng, k, w.dim)
    allcells = np.unique(np.concatenate([c.reshape(-1) for c, _ in cones.values()]))
    f0, g0, l0 = s.get_cells(allcells)
    where = {int(c): j for j, c in enumerate(allcells)}
    if w.schedule is not None:
        for face, fv in w.schedule(steps_before).items():
            s.set_face(face, fv)
    s.step(1)
    out = {}
    for l, (cc, offs) in cones.items():
        centres = cc[:, len(offs) // 2]
        f1, g1, _ = s.get_cells(centres)
        ref_f, ref_g = [], []
        for m in range(len(cc)):
            j = np.array([where[int(c)] for c in cc[m]])
            rf, rg = advance_cone(o, o.tau(l), offs, f0[:, j].T.copy(), None if g0 is None else g0[:, j].T.copy(),
                                  l0[:, j].T.copy(), lat_c, reach, 1 << l, w.dim)
            ref_f.append(rf)
            ref_g.append(rg)
        ref_f = np.array(ref_f).T
        err = float(np.max(np.abs(f1 - ref_f)) / np.max(np.abs(ref_f)))
        if g0 is not None:
            ref_g = np.array(ref_g).T
            err = max(err, float(np.max(np.abs(g1 - ref_g)) / np.max(np.abs(ref_g))))
        out[l] = err
    say(f"[fullsize] {w.name} {storage}: {s.n} cells, sampled {k} cones per level, max relative error {out}")
    s.close()
    for l, err in out.items():
        assert err < tol, (l, err)
    return out


def small_twin(w):
    """a small grid of the same lattice and level count, for the oracle's
    single-cell collisions and relaxation times (the grid itself is unused)"""
    if w.name == "sphere":
        return W.sphere(scale=8)
    if w.name == "airfoil":
        return W.airfoil(scale=16)
    if w.name == "cylinder":
        return W.cylinder(scale=16)
    raise ValueError(w.name)


# tolerances: FP32 collisions round at 2^-24 per operation, some 40
# operations per population and step, up to 4 substeps -> 1e-5 of max |f|;
# FP16 storage of f - w rounds at 2^-11 of |f - w| -> 2e-3
@pytest.mark.parametrize("storage,tol", [("fp32", 1e-5), ("fp16", 2e-3)])
def test_sphere_full_size_sampled(storage, tol):
    """512 x 256 x 256 coarse, three levels (64.7 M cells): coarse and finest
    bulk cells after one coarse step (1 and 4 substeps)."""
    sampled_check(W.sphere(storage=storage), storage, levels=[0, 2], k=24, tol=tol)


def test_cylinder_full_size_sampled():
    """1024 x 512 coarse, four levels: every level (1 to 8 substeps)."""
    sampled_check(W.cylinder(), "fp32", levels=[0, 1, 2, 3], k=12, tol=1e-5)


def test_airfoil_full_size_sampled():
    """2048 x 1024 coarse, three levels, D2Q21 Newton with warm start and the
    shock sensor: coarse and fine bulk cells (1 and 4 substeps)."""
    sampled_check(W.airfoil(), "fp32", levels=[0, 2], k=8, tol=2e-5, steps_before=5)
