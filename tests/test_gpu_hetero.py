"""GPU parity of host + GPU co-execution (section 5), through the C ABI: the
lattice split between host cores (m border columns per side) and the GPU,
halos swapped every step, against the CPU oracle.

Bar: per population relative to its weight, max |f - f_ref| / w_l <= 1e-12
(FP64; the host part and the GPU part round differently)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1703_04594_amd import inputs
from paper_1703_04594_amd.lbm import Hetero, Lattice

from _util import G, TAU, TB, TT, WC, oracle_window_site, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relw(a, b):
    return float(np.max(np.abs(a - b) / WC))


def random_state(lx, ly, seed, amp=0.05):
    return WC * (1.0 + amp * inputs.population_noise(lx, ly, seed))


@pytest.mark.parametrize("ybc", ["walls", "periodic"])
@pytest.mark.parametrize("lx,m", [(40, 0), (40, 2), (40, 5), (40, 17), (41, 19)])
def test_split_lattice_matches_oracle(ybc, lx, m):
    ly, g = 30, -1e-3                 # (41, 19): the GPU keeps 3 columns, the least allowed
    say(f"hetero {ybc} lx={lx} m={m}")
    f0 = random_state(lx, ly, 21)
    h = Hetero(lx, ly, TAU, g, TB, TT, ybc=ybc, m=m, host_threads=4, device=DEV)
    h.set_pops(f0)
    assert np.array_equal(h.get_pops(), f0)
    ref = oracle.RefLattice(lx, ly, TAU, g, TB, TT, ybc=oracle.WALL if ybc == "walls" else oracle.PERIODIC)
    ref.set_pops(f0)
    for n in (1, 4):                   # after 1 and 5 steps
        h.step(n)
        ref.step(n)
        err = relw(h.get_pops(), ref.get_pops())
        assert err <= 1e-12, (ybc, m, err)
    t = h.times()
    assert t["wall"] > 0 and t["gpu"] > 0
    if m:
        assert t["host"] > 0 and t["swap"] > 0
    h.close()


def test_split_2048x4096_rt():
    """The benchmark lattice and split: RT state, m = 64, 20 steps.  The
    whole lattice against the GPU-only step (itself pinned to the oracle),
    and sites on both seams against windowed oracle runs."""
    lx, ly, m, n = 2048, 4096, 64, 20
    say("hetero 2048x4096 m=64")
    P = inputs.rt_perturbation(lx, ly, 1)
    lat = Lattice(lx, ly, TAU, G, TB, TT, step="fused", device=DEV)
    lat.init_rt(torch.tensor(P, device=DEV))
    f0 = lat.get_pops().cpu().numpy()
    lat.step(n)
    want = lat.get_pops().cpu().numpy()
    del lat
    torch.cuda.empty_cache()
    h = Hetero(lx, ly, TAU, G, TB, TT, m=m, host_threads=16, device=DEV)
    h.set_pops(f0)
    del f0
    h.step(n)
    got = h.get_pops()
    h.close()
    err = relw(got, want)
    assert err <= 1e-12, err
    for x0 in (m - 3, m - 1, m, m + 2, lx - m - 3, lx - m - 1, lx - m, lx - m + 2, 0, lx - 1):
        for y0 in (0, 2, ly // 2, ly - 1):
            ref = oracle_window_site(P, lx, ly, x0, y0, n)
            e = float(np.max(np.abs(got[:, x0, y0] - ref) / WC[:, 0, 0]))
            assert e <= 1e-12, (x0, y0, e)


def test_split_beyond_16_bit_columns():
    """A lattice wider than 32767 columns: the halo messages name GPU
    columns past the 16-bit range.  The whole lattice against the GPU-only
    step after 3 steps."""
    lx, ly, m, n = 40000, 12, 3, 3
    say("hetero 40000x12 m=3")
    f0 = random_state(lx, ly, 23)
    lat = Lattice(lx, ly, TAU, -1e-3, TB, TT, step="fused", device=DEV)
    lat.set_pops(torch.tensor(f0, device=DEV))
    lat.step(n)
    want = lat.get_pops().cpu().numpy()
    del lat
    torch.cuda.empty_cache()
    h = Hetero(lx, ly, TAU, -1e-3, TB, TT, m=m, host_threads=4, device=DEV)
    h.set_pops(f0)
    h.step(n)
    got = h.get_pops()
    h.close()
    err = relw(got, want)
    assert err <= 1e-12, err
