"""CPU tests of liblbm.so: it loads and exports every entry point of
include/lbm.h, its host grid builder matches the oracle's bit for bit, both
reject the same inconsistent masks, and host-only contexts refuse device
work.  No compute call reaches a GPU here."""
import os
import re
import subprocess

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W
from edge_cases import edge_cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)) - {"lbm_dev_alloc_fn", "lbm_dev_free_fn"})


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    syms = header_symbols()
    assert sorted(B.EXPORTS) == syms
    for s in syms:
        assert hasattr(lib, s), s
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lbm_\w+)", out))
    assert set(syms) <= exported


def cases():
    out = [("cavity", W.cavity(n=16, steps=1)), ("cavity64", W.cavity(n=64, steps=1)),
           ("shear3", W.shear(n=16, levels=3, steps=1)), ("cyl", W.cylinder(scale=16, steps=1)),
           ("sod", W.sod(nx=128, ny=8, steps=1)), ("airfoil", W.airfoil(scale=16, steps=1)),
           ("sphere", W.sphere(scale=8, steps=1))]
    w = W.shear(n=24, levels=2, steps=1)
    m = np.zeros((24, 24), np.uint8)
    m[6:18, 4:20] = 1
    m[10:14, 2:4] = 1
    w.refine = [W.Mask(m[4:20, 0:22].copy(), (0, 4))]
    w.refine[0].data[:] = m[4:20, 0:22]
    w.faces = [W.Face("wall"), W.Face("wall"), W.Face("periodic"), W.Face("periodic"), W.Face(), W.Face()]
    out.append(("blob", w))
    # two ghost layers at the interfaces (largest velocity component 2)
    out.append(("shear_q13", W.shear(n=32, levels=3, lattice="D2Q13", collision="DDF_NEWTON", T0=0.35)))
    return out + edge_cases()


@pytest.mark.parametrize("name,w", cases(), ids=[c[0] for c in cases()])
def test_host_grid_matches_oracle_bit_exactly(name, w):
    o = Oracle.from_workload(w)
    ref = o.export()
    s = B.LBM.from_workload(w, storage="fp64" if w.collision != "DDF_NEWTON" else "fp32", host_only=True)
    got = s.export()
    assert s.n == o.n
    assert list(s.n_per_level) == list(o.level_counts())
    for k in ["coords", "level", "flags", "nbr", "child", "bc_src"]:
        assert ref[k].shape == got[k].shape, k
        assert np.array_equal(ref[k], got[k]), k
    assert abs(s.eq_fine - B.equivalent_fine_cells(o.level_counts())) < 1e-9


def test_mask_errors_agree():
    bad = [W.shear(n=16, levels=3, steps=1, band=[(0.5, 1.0), (0.5, 0.75)])]
    w = W.shear(n=16, levels=3, steps=1)
    r1 = np.ones((4, 32), np.uint8)
    w.refine[1] = W.Mask(r1, (0, 0))
    bad.append(w)
    w = W.cavity(n=16, steps=1)
    w.faces[1] = W.Face("periodic")  # unpaired periodic face
    bad.append(w)
    for w in bad:
        with pytest.raises(RuntimeError):
            Oracle.from_workload(w)
        with pytest.raises(B.LbmError) as e:
            B.LBM.from_workload(w, host_only=True)
        assert e.value.code == -2


def test_host_only_context_refuses_device_work():
    w = W.cavity(n=16, steps=1)
    s = B.LBM.from_workload(w, host_only=True)
    with pytest.raises(B.LbmError) as e:
        s.init(np.zeros((3, s.n)))
    assert e.value.code == -5
    with pytest.raises(B.LbmError) as e:
        s.step(1)
    assert e.value.code == -5


def test_unsupported_combinations_rejected():
    with pytest.raises(B.LbmError) as e:
        B.LBM("D2Q37", "RR", "fp32", host_only=True)
    assert e.value.code == -7
    with pytest.raises(B.LbmError):
        B.LBM("D2Q21", "DDF_NEWTON", "fp16", host_only=True)
    with pytest.raises(B.LbmError):
        B.LBM("D2Q13", "DDF_POLY", "fp32", host_only=True)


def test_equivalent_fine_cells_paper_table():
    """Sec. 7.3 table: equivalent fine cells = sum n_i / 2^i (paper numbering,
    i = 0 finest), printed rounded down."""
    path = os.path.join(ROOT, "tests", "golden", "aeolian_grid_levels.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        left, total, eq = line.split("|")
        nums = [int(x) for x in left.split()[1:]]
        coarse_first = nums[::-1]  # library numbering: level 0 coarsest
        assert sum(nums) == int(total)
        assert int(B.equivalent_fine_cells(coarse_first)) == int(eq)


@pytest.mark.parametrize("name,w", cases(), ids=[c[0] for c in cases()])
def test_brick_layout_counts(name, w):
    """Device placement: slots come in whole 64-slot bricks per level, every
    cell has one, and every ghost / boundary-layer cell keeps an explicit
    row of pull sources (the brick arithmetic covers bulk cells only)."""
    s = B.LBM.from_workload(w, host_only=True)
    lay = s.layout()
    assert lay["slots"] % 64 == 0 and sum(lay["slots_per_level"]) == lay["slots"]
    assert all(v % 64 == 0 for v in lay["slots_per_level"])
    assert all(sl >= n for sl, n in zip(lay["slots_per_level"], s.n_per_level))
    e = s.export()
    lev, flags = e["level"], e["flags"]
    special = (flags & 0x0F) != 0  # coarse ghost, fine ghost, Neumann, equilibrium layer
    for l in range(s.n_levels):
        assert lay["rows_per_level"][l] >= int(np.count_nonzero(special & (lev == l)))
        assert lay["rows_per_level"][l] <= int(s.n_per_level[l])


def test_brick_layout_uniform_periodic_needs_no_rows():
    """On a periodic uniform grid whose extent is a whole number of bricks
    every cell is a bulk cell; with an extent that is not, only cells within
    the lattice reach of the wrap need rows."""
    s = B.LBM.from_workload(W.shear(n=32, levels=1, steps=1), host_only=True)
    assert s.layout()["exception_rows"] == 0
    s = B.LBM.from_workload(W.shear(n=20, levels=1, steps=1), host_only=True)
    rows = s.layout()["exception_rows"]
    # wrap columns / rows: the last brick is half empty, so cells within one
    # cell of the wrap in x or y take rows: 20 * 20 - 18 * 18 = 76
    assert rows == 20 * 20 - 18 * 18


def test_in_place_streaming_limits():
    """in-place streaming is accepted on refined grids with any faces
    (boundary layers are filled in the level's phase) and refused for the
    multiplier surrogate"""
    w = W.shear(n=16, levels=2, lattice="D2Q9", collision="RR")
    s = B.LBM.from_workload(w, host_only=True, in_place=True)
    assert s.n_levels == 2
    s = B.LBM.from_workload(W.cylinder(scale=16, steps=1), host_only=True, in_place=True)
    assert s.n_levels == 4
    w = W.airfoil(scale=16, steps=1)
    w.collision = "DDF_MLP"
    with pytest.raises(B.LbmError) as e:
        B.LBM.from_workload(w, host_only=True, in_place=True)
    assert e.value.code == -7
    s = B.LBM.from_workload(W.cavity(n=16, levels=1), host_only=True, in_place=True)
    assert s.n == 256


@pytest.mark.parametrize("name,w", [c for c in cases() if c[0] in ("cyl", "sphere", "ragged3d", "sod")],
                         ids=["cyl", "sphere", "ragged3d", "sod"])
def test_layout_export_is_consistent(name, w):
    """lbm_layout_export on a host-built grid: every cell owns one slot of
    its level's range, the exception rows are numbered brick by brick in
    lane order, and the masks count them"""
    s = B.LBM.from_workload(w, host_only=True)
    info = s.layout()
    d = s.layout_export()
    slot = d["slot_of"].astype(np.int64)
    assert len(np.unique(slot)) == s.n and slot.min() >= 0 and slot.max() < info["slots"]
    lev = s.export(("level",))["level"]
    bounds = np.concatenate([[0], np.cumsum(info["slots_per_level"])])
    assert np.all(slot >= bounds[lev]) and np.all(slot < bounds[lev + 1])
    rows = d["xrow_of"]
    has = rows >= 0
    assert has.sum() == info["exception_rows"]
    assert np.array_equal(np.sort(rows[has]), np.arange(info["exception_rows"]))
    bits = np.array([bin(int(v)).count("1") for v in d["xmask"]])
    assert bits.sum() == info["exception_rows"]
    # rows follow the slots of their cells
    order = np.argsort(slot[has])
    assert np.all(np.diff(rows[has][order]) > 0)
    s.close()
