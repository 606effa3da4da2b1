"""The host-core step (the host part of host + GPU co-execution, section 5)
against the CPU oracle, and the co-execution entry points' host-side
validation.  CPU only: nothing here reaches a GPU.

Bar: per population relative to its weight, max |f_host - f_ref| / w_l <=
1e-12 after a few steps (FP64 on both sides, different rounding order)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1703_04594_amd import inputs, lbm

from _util import TAU, TB, TT, WC


def relw(a, b):
    return float(np.max(np.abs(a - b) / WC))


def random_state(lx, ly, seed, amp=0.05):
    return WC * (1.0 + amp * inputs.population_noise(lx, ly, seed))


@pytest.mark.parametrize("ybc", ["walls", "periodic"])
@pytest.mark.parametrize("lx,ly", [(13, 37), (9, 64)])
def test_host_step_matches_oracle(ybc, lx, ly):
    g = -1e-3
    f0 = random_state(lx, ly, 11)
    host = lbm.HostLattice(lx, ly, TAU, g, TB, TT, ybc=ybc, threads=2)
    host.set_pops(f0)
    assert np.array_equal(host.get_pops(), f0)
    ref = oracle.RefLattice(lx, ly, TAU, g, TB, TT, ybc=oracle.WALL if ybc == "walls" else oracle.PERIODIC)
    ref.set_pops(f0)
    for n in (1, 2, 2):          # after 1, 3 and 5 steps
        host.step(n)
        ref.step(n)
        err = relw(host.get_pops(), ref.get_pops())
        assert err <= 1e-12, (ybc, lx, ly, err)


@pytest.mark.parametrize("tau", [0.505, 2.5])
def test_host_step_relaxation_extremes(tau):
    lx, ly = 11, 29
    f0 = random_state(lx, ly, 13, amp=0.02)
    host = lbm.HostLattice(lx, ly, tau, -1e-4, TB, TT, threads=2)
    host.set_pops(f0)
    host.step(10)
    ref = oracle.RefLattice(lx, ly, tau, -1e-4, TB, TT)
    ref.set_pops(f0)
    ref.step(10)
    assert relw(host.get_pops(), ref.get_pops()) <= 1e-12


def test_host_zero_steps_change_nothing():
    lx, ly = 9, 16
    f0 = random_state(lx, ly, 14)
    host = lbm.HostLattice(lx, ly, TAU, 0.0, TB, TT)
    host.set_pops(f0)
    host.step(0)
    assert np.array_equal(host.get_pops(), f0)


def test_host_step_is_independent_of_the_thread_count():
    lx, ly = 16, 45
    f0 = random_state(lx, ly, 12)
    outs = []
    for threads in (1, 3, 8):
        host = lbm.HostLattice(lx, ly, TAU, -1e-5, TB, TT, threads=threads)
        host.set_pops(f0)
        host.step(4)
        outs.append(host.get_pops())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_co_execution_arguments_are_validated_on_the_host():
    L = lbm.lib()
    p = lbm.make_params(64, 48, TAU)
    w0 = L.lbm_hetero_workspace_bytes(ctypes.byref(p), 0)
    assert w0 == lbm.workspace_bytes(lbm.make_params(64, 48, TAU, step="fused"))
    # m columns per side on the host: the GPU part is 64 - 2m + 6 columns wide
    assert L.lbm_hetero_workspace_bytes(ctypes.byref(p), 8) == \
        lbm.workspace_bytes(lbm.make_params(54, 48, TAU, step="fused"))
    for m in (1, -1, 31, 32):    # m >= 2 and lx - 2m >= 3
        assert L.lbm_hetero_workspace_bytes(ctypes.byref(p), m) == 0, m
    p32 = lbm.make_params(64, 48, TAU, precision="fp32")
    assert L.lbm_hetero_workspace_bytes(ctypes.byref(p32), 8) == 0
    assert L.lbm_host_lattice_bytes(ctypes.byref(p32)) == 0
    h = ctypes.c_void_p()
    assert L.lbm_hetero_create(ctypes.byref(p), 1, 4, ctypes.c_void_p(4096), 1 << 30, None, ctypes.byref(h)) == 1
    assert b"m must be" in L.lbm_hetero_last_error(None)
    assert L.lbm_hetero_create(ctypes.byref(p), 8, 0, ctypes.c_void_p(4096), 1 << 30, None, ctypes.byref(h)) == 1
    assert not h.value
    buf = np.zeros(8)
    assert L.lbm_host_step(ctypes.byref(p), buf.ctypes.data, buf.ctypes.data, 1, 1) == 1
    assert L.lbm_host_step(ctypes.byref(p), buf.ctypes.data, None, 1, 1) == 1


def draw_host_cases(n, seed=20170317):
    rng = np.random.default_rng(seed)
    return [dict(lx=int(rng.integers(7, 60)), ly=int(rng.integers(7, 140)), tau=float(rng.uniform(0.52, 2.0)),
                 g=float(rng.uniform(-1e-3, 1e-3)), tb=float(rng.uniform(0.7, 1.5)), tt=float(rng.uniform(0.7, 1.5)),
                 ybc=str(rng.choice(["walls", "periodic"])), threads=int(rng.integers(1, 5)),
                 n=int(rng.integers(1, 6)), seed=900 + i) for i in range(n)]


@pytest.mark.parametrize("case", draw_host_cases(24), ids=[str(i) for i in range(24)])
def test_host_step_random_configuration(case):
    """Seeded random shapes (ragged against the 8-row blocks), relaxation
    times, gravity, wall temperatures, boundaries and thread counts."""
    c = case
    f0 = random_state(c["lx"], c["ly"], c["seed"], amp=0.02)
    host = lbm.HostLattice(c["lx"], c["ly"], c["tau"], c["g"], c["tb"], c["tt"], ybc=c["ybc"], threads=c["threads"])
    host.set_pops(f0)
    host.step(c["n"])
    ref = oracle.RefLattice(c["lx"], c["ly"], c["tau"], c["g"], c["tb"], c["tt"],
                            ybc=oracle.WALL if c["ybc"] == "walls" else oracle.PERIODIC)
    ref.set_pops(f0)
    ref.step(c["n"])
    err = relw(host.get_pops(), ref.get_pops())
    assert err <= 1e-12, (c, err)
