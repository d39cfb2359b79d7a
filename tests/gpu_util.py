"""Helpers shared by the GPU parity tests: run a workload on the HIP library
and on the oracle from the same seeded inputs, and compare the macroscopic
fields with the volume-weighted relative L2 norm."""
import sys

import numpy as np

from oracle.oracle import Oracle
from paper_2504_04465_amd import lbm as B


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(q, ref, vol):
    ok = ~np.isnan(ref)
    num = np.sqrt(np.sum(vol[ok] * (q[ok] - ref[ok]) ** 2))
    den = np.sqrt(np.sum(vol[ok] * ref[ok] ** 2))
    return float(num / den) if den > 0 else float(num)


def compare(m_gpu, m_ref, level, dim):
    """relative L2 of rho, of rho - mean(rho), of the velocity vector and
    (DDF) of T; volumes 2^(-D l)."""
    vol = 0.5 ** (dim * level.astype(np.float64))
    ok = ~np.isnan(m_ref[0])
    assert np.array_equal(np.isnan(m_gpu[0]), ~ok), "fine-ghost NaN pattern differs"
    out = {"rho": rel_l2(m_gpu[0], m_ref[0], vol)}
    rbar = np.sum(vol[ok] * m_ref[0][ok]) / np.sum(vol[ok])
    out["drho"] = rel_l2(m_gpu[0] - rbar, m_ref[0] - rbar, vol)
    du = np.concatenate([m_gpu[1 + d][ok] - m_ref[1 + d][ok] for d in range(dim)])
    uu = np.concatenate([m_ref[1 + d][ok] for d in range(dim)])
    vv = np.concatenate([vol[ok]] * dim)
    out["u"] = float(np.sqrt(np.sum(vv * du ** 2)) / max(np.sqrt(np.sum(vv * uu ** 2)), 1e-300))
    if m_ref.shape[0] > 1 + dim:
        out["T"] = rel_l2(m_gpu[1 + dim], m_ref[1 + dim], vol)
    # worst single cell, relative to the largest value of the field, so that a
    # wrong corner or interface cell cannot hide in the volume-weighted norm
    out["rho_max"] = float(np.max(np.abs(m_gpu[0][ok] - m_ref[0][ok])) / np.max(np.abs(m_ref[0][ok])))
    dun = np.sqrt(sum((m_gpu[1 + d][ok] - m_ref[1 + d][ok]) ** 2 for d in range(dim)))
    un = np.sqrt(sum(m_ref[1 + d][ok] ** 2 for d in range(dim)))
    out["u_max"] = float(np.max(dun) / max(np.max(un), 1e-300))
    if m_ref.shape[0] > 1 + dim:
        out["T_max"] = float(np.max(np.abs(m_gpu[1 + dim][ok] - m_ref[1 + dim][ok])) / np.max(np.abs(m_ref[1 + dim][ok])))
    return out


def assert_within(err, tol, tol_rho=None, cell=10.0):
    """relative L2 of u and rho within their bounds, and the worst cell within
    `cell` times the bound (relative to the field's largest value)"""
    tr = tol if tol_rho is None else tol_rho
    assert err["u"] <= tol and err["rho"] <= tr, err
    assert err["u_max"] <= cell * tol and err["rho_max"] <= cell * tr, err
    if "T" in err:
        assert err["T"] <= tr and err["T_max"] <= cell * tr, err


def run_pair(w, steps, storage, oracle_over=None, lib_over=None, schedule=True):
    """same workload, same seeded initial moments, `steps` coarse steps on
    both sides; returns (gpu moments, oracle moments, levels, gpu handle)."""
    o = Oracle.from_workload(w, **(oracle_over or {}))
    s = B.LBM.from_workload(w, storage=storage, **(lib_over or {}))
    e = o.export()
    coords, level = s.coords_levels()
    assert np.array_equal(coords, e["coords"]) and np.array_equal(level, e["level"])
    m0 = w.initial_moments(coords, level)
    o.init(m0)
    s.init(m0)
    if w.inflow_noise is not None:
        du = w.inflow_noise(coords, level)
        o.set_inflow_noise(du)
        s.set_inflow_noise(du)
    if not (schedule and w.schedule is not None):
        o.step(steps)
        s.step(steps)
    else:
        for k in range(steps):
            for face, f in w.schedule(k).items():
                o.set_face(face, f)
                s.set_face(face, f)
            o.step(1)
            s.step(1)
    return s.moments(), o.moments(), level, s, o
