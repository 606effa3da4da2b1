"""GPU parity of the layout study (the four data layouts of section 4,
Table 2), through the C ABI.

* Placement: every element of a packed buffer sits where the layout's
  definition puts it.  The expected buffers are built here by reshaping and
  transposing the canonical array (y = k M + i split into lane and partition
  row), not by the kernels' index arithmetic.
* propagate is a permutation, so bitwise against the oracle's (periodic in x
  and y) on small lattices with ragged chunks, and bitwise against
  per-population periodic rolls of a tagged lattice at 2160x8192.
* collide is compared with the oracle per population relative to its weight,
  max |f_gpu - f_ref| / w_l <= 1e-13, the bar of the library's own collide;
  at 2160x8192 on 1024 sampled sites.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1703_04594_amd import inputs, lbm
from paper_1703_04594_amd.lbm import Lattice

from _util import TAU, W, WC, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GRAV = -1e-3

CASES = [("aos", 1), ("soa", 1), ("csoa", 1), ("csoa", 8), ("csoa", 32),
         ("caosoa", 1), ("caosoa", 8), ("caosoa", 32)]
FULL = [("aos", 1), ("soa", 1)] + [(lay, vl) for lay in ("csoa", "caosoa") for vl in (8, 16, 32, 64)]


def tagged(lx, ly):
    return (np.arange(37 * lx * ly, dtype=np.float64) + 1.0).reshape(37, lx, ly)


def expected_buffer(layout, vl, canon):
    """The layout's element order, from the canonical (37, lx, ly) array."""
    q, lx, ly = canon.shape
    if layout == "aos":
        return canon.transpose(1, 2, 0).ravel()             # (x, y, l)
    if layout == "soa":
        return canon.ravel()                                 # (l, x, y)
    m = ly // vl
    parts = canon.reshape(q, lx, vl, m)                      # y = k m + i -> (l, x, k, i)
    if layout == "csoa":
        return parts.transpose(0, 1, 3, 2).ravel()           # (l, x, i, k)
    return parts.transpose(1, 3, 0, 2).ravel()               # (x, i, l, k)


def relw(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b) / WC))


@pytest.mark.parametrize("layout,vl", CASES)
def test_placement_and_round_trip(layout, vl):
    lx, ly = 11, 96
    say(f"study placement {layout} vl={vl}")
    t = tagged(lx, ly)
    canon = torch.tensor(t, device=DEV)
    buf = lbm.study_pack(layout, vl, canon)
    assert np.array_equal(buf.cpu().numpy(), expected_buffer(layout, vl, t))
    assert torch.equal(lbm.study_unpack(layout, vl, lx, ly, buf), canon)


@pytest.mark.parametrize("layout,vl,lx,ly", [(lay, vl, 13, 96) for lay, vl in CASES]
                         + [("aos", 1, 37, 200), ("soa", 1, 37, 200), ("csoa", 8, 37, 200),
                            ("caosoa", 8, 37, 200), ("csoa", 64, 9, 192), ("caosoa", 64, 9, 192),
                            # the smallest lattices each layout takes
                            ("aos", 1, 7, 7), ("soa", 1, 7, 7), ("csoa", 2, 7, 8), ("caosoa", 2, 7, 8)])
def test_propagate_is_the_oracle_permutation(layout, vl, lx, ly):
    say(f"study propagate {layout} vl={vl} {lx}x{ly}")
    t = tagged(lx, ly)
    src = lbm.study_pack(layout, vl, torch.tensor(t, device=DEV))
    dst = torch.full_like(src, -1.0)
    lbm.study_propagate(layout, vl, lx, ly, src, dst)
    got = lbm.study_unpack(layout, vl, lx, ly, dst).cpu().numpy()
    ref = oracle.RefLattice(lx, ly, TAU, ybc=oracle.PERIODIC)
    ref.set_pops(t)
    ref.propagate()
    assert np.array_equal(got, ref.get_pops())


def random_state(lx, ly, seed, amp=0.05):
    return WC * (1.0 + amp * inputs.population_noise(lx, ly, seed))


def test_collide_matches_oracle_in_every_layout():
    lx, ly = 13, 96
    say("study collide, all layouts")
    f0 = random_state(lx, ly, 5)
    ref = oracle.RefLattice(lx, ly, TAU, GRAV, ybc=oracle.PERIODIC)
    ref.set_pops(f0)
    ref.collide()
    want = ref.get_pops()
    outs = {}
    for layout, vl in CASES:
        buf = lbm.study_pack(layout, vl, torch.tensor(f0, device=DEV))
        lbm.study_collide(layout, vl, lx, ly, TAU, GRAV, buf)
        got = lbm.study_unpack(layout, vl, lx, ly, buf).cpu().numpy()
        err = relw(got, want)
        assert err <= 1e-13, (layout, vl, err)
        outs[(layout, vl)] = got
    # the site arithmetic is the same in every layout
    base = outs[("soa", 1)]
    for key, got in outs.items():
        assert np.array_equal(got, base), key


def test_full_size_2160x8192():
    """The lattice and layouts that bench.py --layout-study times."""
    lx, ly = 2160, 8192
    ex, ey = lbm.velocity_table()
    say("study 2160x8192: propagate permutation")
    canon = torch.arange(37 * lx * ly, dtype=torch.float64, device=DEV).reshape(37, lx, ly)
    want = torch.stack([torch.roll(canon[l], shifts=(ex[l], ey[l]), dims=(0, 1)) for l in range(37)])
    for layout, vl in FULL:
        say(f"  propagate {layout} vl={vl}")
        src = lbm.study_pack(layout, vl, canon)
        dst = torch.empty_like(src)
        lbm.study_propagate(layout, vl, lx, ly, src, dst)
        del src
        got = lbm.study_unpack(layout, vl, lx, ly, dst)
        del dst
        assert torch.equal(got, want), (layout, vl)
        del got
    del canon, want
    torch.cuda.empty_cache()

    say("study 2160x8192: collide on an RT state")
    lat = Lattice(lx, ly, TAU, -1e-5, 4 / 3, 2 / 3, device=DEV)
    lat.init_rt(torch.tensor(inputs.rt_perturbation(lx, ly, 1), device=DEV))
    lat.step(3)
    f = lat.get_pops()
    del lat
    torch.cuda.empty_cache()
    rng = np.random.default_rng(7)
    xs = torch.tensor(rng.integers(0, lx, 1024), device=DEV)
    ys = torch.tensor(rng.integers(0, ly, 1024), device=DEV)
    sample_in = f[:, xs, ys].cpu().numpy().reshape(37, 8, 128)
    ref = oracle.RefLattice(8, 128, TAU, GRAV, ybc=oracle.PERIODIC)
    ref.set_pops(sample_in)
    ref.collide()
    want = ref.get_pops()
    base = None
    for layout, vl in FULL:
        say(f"  collide {layout} vl={vl}")
        buf = lbm.study_pack(layout, vl, f)
        lbm.study_collide(layout, vl, lx, ly, TAU, GRAV, buf)
        got = lbm.study_unpack(layout, vl, lx, ly, buf)
        del buf
        sample = got[:, xs, ys].cpu().numpy().reshape(37, 8, 128)
        err = float(np.max(np.abs(sample - want) / W[:, None, None]))
        assert err <= 1e-13, (layout, vl, err)
        if base is None:
            base = got
        else:
            assert torch.equal(got, base), (layout, vl)
        del got
