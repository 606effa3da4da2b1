"""Pins of the oracle's lattice constants and equilibrium (CPU only).

Everything here is checked against mathematics the model fixes, not against
the oracle's own formulas: Gaussian moment identities evaluated in exact
rational arithmetic, the symmetry of the hop set, and the closed-form moments
of the Maxwellian that a 4th-order Hermite equilibrium must reproduce.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle


def dfact(i):  # (2i-1)!!
    r = 1
    for k in range(2 * i - 1, 1, -2):
        r *= k
    return r


def test_velocity_set_shape_and_symmetry():
    # 37 hops of length at most 3 (section 3: populations move up to three sites)
    ex, ey = oracle.velocity_table()
    hops = list(zip(ex.tolist(), ey.tolist()))
    assert len(hops) == 37 and len(set(hops)) == 37
    assert max(max(abs(a), abs(b)) for a, b in hops) == 3
    s = set(hops)
    for a, b in hops:
        assert (-a, b) in s and (a, -b) in s and (b, a) in s
    r2 = [a * a + b * b for a, b in hops]
    counts = {k: r2.count(k) for k in sorted(set(r2))}
    assert counts == {0: 1, 1: 4, 2: 4, 4: 4, 5: 8, 8: 4, 9: 4, 10: 8}
    # canonical order: by |e|^2, then angle in [0, 2pi)
    ang = [math.atan2(b, a) % (2 * math.pi) for a, b in hops]
    keys = list(zip(r2, ang))
    assert keys == sorted(keys)
    # halo depth: 15 hops with ex >= 1, 8 with ex >= 2, 3 with ex == 3
    assert sum(a >= 1 for a, _ in hops) == 15
    assert sum(a >= 2 for a, _ in hops) == 8
    assert sum(a >= 3 for a, _ in hops) == 3


def test_quadrature_exact_in_rationals():
    """Sum_l w_l xi_x^(2i) xi_y^(2j) = (2i-1)!!(2j-1)!! for 2i+2j <= 8, with
    the DOUBLE weights and c evaluated exactly as rationals."""
    ex, ey = oracle.velocity_table()
    w = oracle.weights()
    c = Fraction(oracle.scale_c())
    for i in range(5):
        for j in range(5):
            if 2 * i + 2 * j > 8:
                continue
            acc = sum(Fraction(float(wl)) * (c * int(a)) ** (2 * i) * (c * int(b)) ** (2 * j)
                      for wl, a, b in zip(w, ex, ey))
            target = dfact(i) * dfact(j)
            assert abs(float(acc - target)) <= 1e-15 * target, (i, j, float(acc - target))
            # odd moments vanish exactly by symmetry
            odd = sum(Fraction(float(wl)) * (c * int(a)) ** (2 * i + 1) * (c * int(b)) ** (2 * j)
                      for wl, a, b in zip(w, ex, ey))
            assert odd == 0
    # quad-precision residuals of the solve itself
    assert np.all(np.abs(oracle.quadrature_residuals()) < 1e-28)


def test_quadrature_is_degree_nine_only():
    # a degree-9 rule cannot integrate xi_x^10: the 10th moment is off
    ex, _ = oracle.velocity_table()
    w = oracle.weights()
    c = oracle.scale_c()
    m10 = float(np.sum(w * (c * ex) ** 10))
    assert abs(m10 - 945.0) > 1.0


def test_weights_positive_and_rest_state():
    w = oracle.weights()
    assert np.all(w > 0)
    assert abs(w.sum() - 1.0) < 1e-15
    # f^eq at rest, unit temperature and density is the weight vector itself
    assert np.array_equal(oracle.feq(1.0, 0.0, 0.0, 1.0), w)


def gaussian_moment(n, mu, var):
    """E[X^n] for X ~ N(mu, var)."""
    return sum(math.comb(n, 2 * k) * mu ** (n - 2 * k) * var ** k * dfact(k)
               for k in range(n // 2 + 1))


@pytest.mark.parametrize("seed", range(6))
def test_equilibrium_reproduces_maxwellian_moments(seed):
    """A 4th-order Hermite equilibrium on an exact degree-9 rule has the
    Maxwellian's moments up to order 4: p = rho T (perfect gas), the heat
    flux and the 4th-order moments.  Pins every term of the equilibrium."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.6, 1.4)
    ux, uy = rng.uniform(-0.15, 0.15, size=2)
    T = rng.uniform(0.65, 1.35)
    ex, ey = oracle.velocity_table()
    c = oracle.scale_c()
    xi_x, xi_y = c * ex, c * ey
    f = oracle.feq(rho, ux, uy, T)
    for p in range(5):
        for q in range(5 - p):
            got = float(np.sum(f * xi_x ** p * xi_y ** q))
            want = rho * gaussian_moment(p, ux, T) * gaussian_moment(q, uy, T)
            assert abs(got - want) <= 2e-14 * max(1.0, abs(want)), (p, q, got, want)
