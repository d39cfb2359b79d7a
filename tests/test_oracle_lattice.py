"""Pins of the oracle's lattices against the paper's lattice table (App. A.1,
Table "lattices_structure") and against the isotropy (Gaussian-moment)
conditions that define the weights."""
import itertools
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.oracle import Oracle

HERE = os.path.dirname(os.path.abspath(__file__))

# lattice name -> (collision used to build it, velocity groups |xi| pattern -> count,
# highest degree of monomials integrated exactly)
SPEC = {
    "D2Q9": ("BGK", {(0, 0): 1, (1, 0): 4, (1, 1): 4}, 5),
    "D2Q13": ("DDF_NEWTON", {(0, 0): 1, (1, 0): 4, (1, 1): 4, (2, 0): 4}, 5),
    "D2Q21": ("DDF_NEWTON", {(0, 0): 1, (1, 0): 4, (1, 1): 4, (2, 0): 4, (2, 2): 4, (3, 0): 4}, 7),
    "D2Q37": ("DDF_POLY", {(0, 0): 1, (1, 0): 4, (1, 1): 4, (2, 0): 4, (2, 1): 8, (2, 2): 4,
                           (3, 0): 4, (3, 1): 8}, 9),
    "D3Q27": ("BGK", None, 5),
}

# exact rational weights printed in the paper's table (D3Q27: product of the
# D1Q3 weights 2/3, 1/6, 1/6)
PRINTED = {
    "D2Q9": ({(0, 0): Fr(4, 9), (1, 0): Fr(1, 9), (1, 1): Fr(1, 36)}, Fr(1, 3)),
    "D2Q13": ({(0, 0): Fr(36, 96), (1, 0): Fr(8, 96), (1, 1): Fr(6, 96), (2, 0): Fr(1, 96)}, Fr(1, 2)),
    "D2Q21": ({(0, 0): Fr(91, 324), (1, 0): Fr(1, 12), (1, 1): Fr(2, 27), (2, 0): Fr(7, 360),
               (2, 2): Fr(1, 432), (3, 0): Fr(1, 1620)}, Fr(2, 3)),
}


def lattice(name):
    coll = SPEC[name][0]
    return Oracle(name, coll, nu_finest=0.1, T0=1.0)


def gauss_moment(p, var):
    """E[X^p] for X ~ N(0, var)."""
    if p % 2:
        return 0.0
    r = 1.0
    for k in range(1, p, 2):
        r *= k
    return r * var ** (p // 2)


@pytest.mark.parametrize("name", list(SPEC))
def test_velocity_set_and_order(name):
    o = lattice(name)
    c = o.c[:, : o.D]
    # canonical order: rest first, then ascending (|xi|^2, xi_x, xi_y, xi_z)
    keys = [(int((v ** 2).sum()),) + tuple(int(x) for x in o.c[i]) for i, v in enumerate(c)]
    assert keys == sorted(keys)
    assert tuple(o.c[0]) == (0, 0, 0)
    assert len({tuple(v) for v in c}) == o.Q
    if SPEC[name][1] is not None:
        groups = {}
        for v in c:
            a, b = sorted(np.abs(v), reverse=True)
            groups[(int(a), int(b))] = groups.get((int(a), int(b)), 0) + 1
        assert groups == SPEC[name][1]
    else:
        assert o.Q == 27 and set(map(tuple, c)) == set(itertools.product((-1, 0, 1), repeat=3))
    for i in range(o.Q):
        assert np.array_equal(o.c[o.opp[i]], -o.c[i])
    assert o.B == int(np.abs(c).max())


@pytest.mark.parametrize("name", ["D2Q9", "D2Q13", "D2Q21"])
def test_printed_rational_weights(name):
    o = lattice(name)
    wt, cs2 = PRINTED[name]
    assert o.cs2 == float(cs2)
    for i in range(o.Q):
        a, b = sorted(np.abs(o.c[i, :2]), reverse=True)
        assert o.w[i] == float(wt[(int(a), int(b))])


def test_d3q27_product_weights():
    o = lattice("D3Q27")
    w1 = {0: Fr(2, 3), 1: Fr(1, 6), -1: Fr(1, 6)}
    for i in range(o.Q):
        exact = w1[int(o.c[i, 0])] * w1[int(o.c[i, 1])] * w1[int(o.c[i, 2])]
        assert o.w[i] == float(exact)
    assert o.cs2 == 1.0 / 3.0


def test_d2q37_weights_match_printed_table():
    o = lattice("D2Q37")
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "d2q37_weights_printed.txt"))
            if l.strip() and not l.startswith("#")]
    printed = {(int(r[1]), int(r[2])): float(r[4]) for r in rows if r[0] != "cs2"}
    cs2 = [float(r[1]) for r in rows if r[0] == "cs2"][0]
    assert abs(o.cs2 - cs2) < 1e-15
    for i in range(o.Q):
        a, b = sorted(np.abs(o.c[i, :2]), reverse=True)
        # the printed values are the re-solved weights truncated to 15 digits
        assert abs(o.w[i] - printed[(int(a), int(b))]) < 1e-15
    # the printed set itself misses unit sum by ~2e-14; the re-solved one does not
    ptot = sum(printed[(int(sorted(np.abs(v[:2]))[1]), int(sorted(np.abs(v[:2]))[0]))] for v in o.c)
    assert abs(ptot - 1.0) > 1e-15
    assert abs(o.w.sum() - 1.0) < 4e-16


@pytest.mark.parametrize("name", list(SPEC))
def test_isotropy_moments(name):
    """sum_i w_i xi^a = Gaussian moment of variance cs2, for every monomial up
    to the lattice's quadrature degree (the defining property of the weights)."""
    o = lattice(name)
    D, deg = o.D, SPEC[name][2]
    xi = o.c[:, :D].astype(np.float64)
    for powers in itertools.product(range(deg + 1), repeat=D):
        if sum(powers) > deg:
            continue
        mono = np.prod([xi[:, d] ** powers[d] for d in range(D)], axis=0)
        lhs = float((o.w * mono).sum())
        rhs = float(np.prod([gauss_moment(p, o.cs2) for p in powers]))
        assert abs(lhs - rhs) < 2e-14 * max(1.0, abs(rhs)), (powers, lhs, rhs)


def test_d2q13_not_isotropic_at_sixth_order():
    """the degree of D2Q13 is exactly five: its sixth moments miss the
    Gaussian's (sum w xi_x^6 = 168/96 against 15 cs2^3 = 180/96)"""
    o = lattice("D2Q13")
    x = o.c[:, 0].astype(np.float64)
    assert abs((o.w * x ** 6).sum() - 168.0 / 96.0) < 1e-14
    assert abs((o.w * x ** 6).sum() - 15.0 * o.cs2 ** 3) > 0.1
