"""Pins of the oracle's propagate, bc and collide (CPU only).

Each check is fixed by the method itself, independently of how the oracle
writes it: a pull propagate is a permutation (brute-force decode of a tagged
lattice), BGK relaxation towards an equilibrium with the same moments
conserves mass, momentum and energy and has the equilibrium as fixed point,
uniform states stay uniform, gravity by equilibrium shift adds exactly g per
step, and a wall that reflects the density of a resting gas at the wall
temperature is indistinguishable from a mirror-image periodic continuation.
"""
import numpy as np
import pytest

import oracle
from paper_1703_04594_amd import inputs

EX, EY = oracle.velocity_table()
W = oracle.weights()


def feq_field(rho, ux, uy, T):
    rho, ux, uy, T = np.broadcast_arrays(rho, ux, uy, T)
    out = np.empty((37,) + rho.shape)
    for idx in np.ndindex(rho.shape):
        out[(slice(None),) + idx] = oracle.feq(rho[idx], ux[idx], uy[idx], T[idx])
    return out


def tagged(lx, ly):
    return (np.arange(37 * lx * ly, dtype=np.float64) + 1.0).reshape(37, lx, ly)


def decode(code, lx, ly):
    c = code.astype(np.int64) - 1
    return c // (lx * ly), (c // ly) % lx, c % ly


@pytest.mark.parametrize("lx,ly", [(7, 9), (13, 8), (16, 16)])
def test_propagate_is_the_pull_permutation_periodic(lx, ly):
    L = oracle.RefLattice(lx, ly, 0.7, ybc=oracle.PERIODIC)
    L.set_pops(tagged(lx, ly))
    L.propagate()
    l, xs, ys = decode(L.get_pops(), lx, ly)
    li, xi, yi = np.meshgrid(np.arange(37), np.arange(lx), np.arange(ly), indexing="ij")
    assert np.array_equal(l, li)
    assert np.array_equal(xs, (xi - EX[:, None, None]) % lx)
    assert np.array_equal(ys, (yi - EY[:, None, None]) % ly)


def test_propagate_with_walls_leaves_exactly_the_ghost_sourced_slots():
    lx, ly = 9, 11
    L = oracle.RefLattice(lx, ly, 0.7)
    t = tagged(lx, ly)
    L.set_pops(t)
    L.propagate()
    f = L.get_pops()
    ghost = np.isnan(f)
    li, xi, yi = np.meshgrid(np.arange(37), np.arange(lx), np.arange(ly), indexing="ij")
    src_y = yi - EY[:, None, None]
    assert np.array_equal(ghost, (src_y < 0) | (src_y >= ly))
    # 15 + 8 + 3 = 26 ghost-sourced slots per column per wall
    assert ghost[:, 0, :3].sum() == 26 and ghost[:, 0, -3:].sum() == 26
    l, xs, ys = decode(np.where(ghost, 1.0, f), lx, ly)
    ok = ~ghost
    assert np.array_equal(xs[ok], ((xi - EX[:, None, None]) % lx)[ok])
    assert np.array_equal(ys[ok], src_y[ok])


def random_state(lx, ly, seed, amp=0.05):
    return W[:, None, None] * (1.0 + amp * inputs.population_noise(lx, ly, seed))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_collide_conserves_per_site(seed):
    lx, ly = 9, 8
    L = oracle.RefLattice(lx, ly, 0.7, ybc=oracle.PERIODIC)
    f0 = random_state(lx, ly, seed)
    L.set_pops(f0)
    L.collide()
    f1 = L.get_pops()
    c = oracle.scale_c()
    xx, yy = (c * EX)[:, None, None], (c * EY)[:, None, None]
    x2 = xx * xx + yy * yy
    rho0 = f0.sum(0)
    ux, uy = (xx * f0).sum(0) / rho0, (yy * f0).sum(0) / rho0
    T = ((x2 * f0).sum(0) / rho0 - ux * ux - uy * uy) / 2
    d_rho = np.abs(f1.sum(0) - rho0)
    d_j = np.hypot((xx * (f1 - f0)).sum(0), (yy * (f1 - f0)).sum(0))
    d_e = np.abs((x2 * (f1 - f0)).sum(0))
    assert np.all(d_rho <= 1e-13 * rho0)
    assert np.all(d_j <= 1e-13 * rho0 * np.sqrt(T))
    assert np.all(d_e <= 1e-13 * rho0 * (ux * ux + uy * uy + 2 * T))
    # and it did change the state (relaxation happened)
    assert np.abs(f1 - f0).max() > 1e-4


def test_equilibrium_is_a_fixed_point_of_collide():
    lx, ly = 6, 7
    rho = inputs.uniform_field(lx, ly, 3, 0.7, 1.3)
    ux = inputs.uniform_field(lx, ly, 4, -0.1, 0.1)
    uy = inputs.uniform_field(lx, ly, 5, -0.1, 0.1)
    T = inputs.uniform_field(lx, ly, 6, 0.7, 1.3)
    L = oracle.RefLattice(lx, ly, 0.8, ybc=oracle.PERIODIC)
    L.init(rho, ux, uy, T)
    f0 = L.get_pops()
    assert np.allclose(f0, feq_field(rho, ux, uy, T), rtol=0, atol=0)
    L.collide()
    # rounding only: relative to the population's own size (|f| reaches several
    # w_l on the outer shells at |u| = 0.1, T = 1.3)
    scale = np.maximum(np.abs(f0), W[:, None, None])
    assert np.max(np.abs(L.get_pops() - f0) / scale) <= 1e-14


def test_uniform_states_stay_uniform():
    """Every site does the same arithmetic on the same inputs, so a uniform
    state stays bitwise uniform along x (and along y when periodic; wall rows
    round their products in another order); in time it moves only by rounding
    (at most 1e-14 w_l per step)."""
    n = 15
    cases = [oracle.RefLattice(8, 9, 0.7, ybc=oracle.PERIODIC),     # periodic, moving, warm
             oracle.RefLattice(8, 9, 0.7, 0.0, 0.8, 0.8)]           # walls, at rest at T_wall
    states = [(1.1, 0.03, -0.02, 1.07), (1.2, 0.0, 0.0, 0.8)]
    for L, st in zip(cases, states):
        L.init(*st)
        f0 = L.get_pops()
        L.step(n)
        f = L.get_pops()
        assert np.all(f == (f[:, :1, :1] if L is cases[0] else f[:, :1, :]))
        assert np.max(np.abs(f - f0) / W[:, None, None]) <= n * 1e-14


def test_gravity_adds_g_per_step():
    """Equilibrium shift u* = u + tau g, T* = T + tau(1-tau)g^2/2: a uniform
    periodic gas gains exactly g per step, keeping rho and T."""
    g = -1e-3
    L = oracle.RefLattice(7, 7, 0.7, g, ybc=oracle.PERIODIC)
    L.init(1.1, 0.0, 0.0, 0.95)
    n = 5
    L.step(n)
    rho, ux, uy, T = L.macros()
    assert np.max(np.abs(rho - 1.1)) <= 1e-14
    assert np.max(np.abs(ux)) <= 1e-15
    assert np.max(np.abs(uy - n * g)) <= 1e-14
    assert np.max(np.abs(T - 0.95)) <= 1e-14


@pytest.mark.parametrize("g", [0.0, -1e-3])
def test_wall_equals_mirror_continuation_for_resting_gas(g):
    """For a gas at rest at the wall temperature with any density field, one
    step with walls equals one step of the periodic lattice of twice the height
    that holds the field and its mirror image (rows -1-k <-> k)."""
    lx, ly, Tw = 12, 10, 0.9
    rho = inputs.uniform_field(lx, ly, 11, 0.8, 1.2)
    L = oracle.RefLattice(lx, ly, 0.7, g, Tw, Tw)
    L.init(rho, 0.0, 0.0, Tw)
    L.step(1)
    rho2 = np.concatenate([rho, rho[:, ::-1]], axis=1)
    P = oracle.RefLattice(lx, 2 * ly, 0.7, g, ybc=oracle.PERIODIC)
    P.init(rho2, 0.0, 0.0, Tw)
    P.step(1)
    a = L.get_pops()
    b = P.get_pops()[:, :, :ly]
    assert np.max(np.abs(a - b) / W[:, None, None]) <= 1e-14


def rt_lattice(lx, ly, seed, tau=0.7, g=-1e-5, xbc=oracle.PERIODIC, ybc=oracle.WALL):
    P = inputs.rt_perturbation(lx, ly, seed)
    y = np.arange(ly)[None, :]
    T0 = 1.0 - np.tanh((y - (ly - 1) / 2 - P) / 2.0) / 3.0
    rho0 = (8.0 / 9.0) / T0
    L = oracle.RefLattice(lx, ly, tau, g, 4 / 3, 2 / 3, xbc=xbc, ybc=ybc)
    L.init(rho0, 0.0, 0.0, T0)
    return L, rho0, T0


def test_open_window_reproduces_the_full_lattice_cone():
    """Sampled full-size parity evolves only a window around each sample with
    open sides; after n steps everything farther than 3n from an open side is
    bitwise the full lattice's."""
    lx, ly, n = 40, 30, 3
    full, rho0, T0 = rt_lattice(lx, ly, 7)
    full.step(n)
    ref = full.get_pops()
    # x window, full height with both walls
    x0, x1 = 10, 30
    win = oracle.RefLattice(x1 - x0, ly, 0.7, -1e-5, 4 / 3, 2 / 3, xbc=oracle.OPEN)
    win.init(rho0[x0:x1], 0.0, 0.0, T0[x0:x1])
    win.step(n)
    got = win.get_pops()
    assert np.array_equal(got[:, 3 * n:-3 * n], ref[:, x0 + 3 * n:x1 - 3 * n])
    # y window touching the bottom wall, open on top
    y1 = 20
    win = oracle.RefLattice(lx, y1, 0.7, -1e-5, 4 / 3, 2 / 3, ybc=(oracle.WALL, oracle.OPEN))
    win.init(rho0[:, :y1], 0.0, 0.0, T0[:, :y1])
    win.step(n)
    assert np.array_equal(win.get_pops()[:, :, :y1 - 3 * n], ref[:, :, :y1 - 3 * n])


def test_openmp_build_is_bitwise_serial():
    a, _, _ = rt_lattice(33, 21, 2)
    b = oracle.RefLattice(33, 21, 0.7, -1e-5, 4 / 3, 2 / 3, openmp=True)
    b.set_pops(a.get_pops())
    a.step(4)
    b.step(4)
    assert np.array_equal(a.get_pops(), b.get_pops())


def test_invalid_parameters_are_rejected():
    with pytest.raises(ValueError):
        oracle.RefLattice(8, 8, 0.5)
    with pytest.raises(ValueError):
        oracle.RefLattice(8, 5, 0.7)       # walls need ly >= 7
    with pytest.raises(ValueError):
        oracle.RefLattice(0, 8, 0.7)
