"""The allocation-free conserved sums (lbm_sums_device) against the
allocating read-back (lbm_stats_get) through the C-ABI: bit-identical
results on two calls in a row on one GPU, the second on a smaller grid (so
stale partials of the first call must not leak into the second), each
into a device buffer allocated by the test before the call."""
import numpy as np
import pytest
import torch

from gpu_util import say
from paper_2504_04465_amd import lbm as B
from paper_2504_04465_amd import workloads as W

pytestmark = pytest.mark.gpu


def check(s, name):
    out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.sums_device(out.data_ptr())
    s.sync()
    got = out.cpu().numpy()
    st = s.stats()
    mom = list(st["momentum"]) + [0.0] * (3 - len(st["momentum"]))
    ref = np.array([st["mass"]] + mom + [st["energy"], st["kinetic_energy"]])
    say(f"[no-alloc] {name}: {got.tolist()}")
    assert np.array_equal(got, ref), (got, ref)
    assert np.isfinite(got).all() and got[0] > 0 and got[5] > 0


def test_sums_device_matches_stats_on_two_grids():
    big = W.sphere(scale=8, steps=2)
    a = B.LBM.from_workload(big, storage="fp32")
    a.init_workload(big)
    a.step(2)
    check(a, "sphere/8 fp32")  # 3 levels, several partial blocks per level
    small = W.cavity(n=16, steps=3)
    b = B.LBM.from_workload(small, storage="fp64")
    b.init_workload(small)
    b.step(3)
    check(b, "cavity16 fp64")  # 2 levels, one block per level
    check(a, "sphere/8 fp32 again")
    a.close()
    b.close()
