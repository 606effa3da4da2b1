"""GPU parity over randomly drawn configurations: lattice shape, relaxation
time, gravity, wall temperatures, y boundary, x mode, step kind, layout and
storage precision, each combination against the CPU oracle after a few steps
from a random near-equilibrium state.  The draws come from one fixed seed, so
the set of cases is the same on every run.

Bars as in the other forward tests: FP64 per population relative to its
weight, max |f - f_ref| / w_l <= 1e-12; FP32-shifted per field against the
FP64 oracle, relative rho and T and absolute u <= 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1703_04594_amd import inputs
from paper_1703_04594_amd.lbm import Lattice

from _util import WC, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def draw_cases(n, seed=20170313):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(n):
        cases.append(dict(
            lx=int(rng.integers(7, 161)), ly=int(rng.integers(7, 601)),
            tau=float(rng.uniform(0.52, 2.0)), g=float(rng.uniform(-1e-3, 1e-3)),
            tb=float(rng.uniform(0.7, 1.5)), tt=float(rng.uniform(0.7, 1.5)),
            ybc=str(rng.choice(["walls", "periodic"])), xmode=str(rng.choice(["wrap", "halo"])),
            step=str(rng.choice(["split", "fused"])), layout=str(rng.choice(["columns", "planes"])),
            precision="fp32" if rng.random() < 0.25 else "fp64", n=int(rng.integers(1, 7)),
            seed=100 + i))
    return cases


CASES = draw_cases(40)


@pytest.mark.parametrize("case", CASES, ids=[f"{i}" for i in range(len(CASES))])
def test_random_configuration_matches_oracle(case):
    c = case
    say(f"random case {c}")
    lx, ly = c["lx"], c["ly"]
    f0 = WC * (1.0 + 0.02 * inputs.population_noise(lx, ly, c["seed"]))
    ref = oracle.RefLattice(lx, ly, c["tau"], c["g"], c["tb"], c["tt"],
                            ybc=oracle.WALL if c["ybc"] == "walls" else oracle.PERIODIC)
    ref.set_pops(f0)
    ref.step(c["n"])
    lat = Lattice(lx, ly, c["tau"], c["g"], c["tb"], c["tt"], precision=c["precision"], ybc=c["ybc"],
                  xmode=c["xmode"], step=c["step"], layout=c["layout"], device=DEV)
    if c["precision"] == "fp64":
        lat.set_pops(torch.tensor(f0, device=DEV))
        lat.step(c["n"])
        err = float(np.max(np.abs(lat.get_pops().cpu().numpy() - ref.get_pops()) / WC))
        assert err <= 1e-12, (c, err)
    else:
        lat.set_pops(torch.tensor(f0 - WC, dtype=torch.float32, device=DEV))
        lat.step(c["n"])
        rho, ux, uy, T = (t.cpu().numpy() for t in lat.macros())
        r_rho, r_ux, r_uy, r_T = ref.macros()
        e_rho = float(np.max(np.abs(rho - r_rho) / r_rho))
        e_T = float(np.max(np.abs(T - r_T) / r_T))
        e_u = float(max(np.max(np.abs(ux - r_ux)), np.max(np.abs(uy - r_uy))))
        assert e_rho <= 1e-5 and e_T <= 1e-5 and e_u <= 1e-5, (c, e_rho, e_T, e_u)
    lat.close()


def draw_study_cases(n, seed=20170314):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(n):
        layout = str(rng.choice(["aos", "soa", "csoa", "caosoa"]))
        vl = 1 if layout in ("aos", "soa") else int(2 ** rng.integers(0, 7))
        m = int(rng.integers(3, max(4, 400 // vl)))
        cases.append(dict(layout=layout, vl=vl, lx=int(rng.integers(7, 90)), ly=vl * max(m, -(-7 // vl)),
                          tau=float(rng.uniform(0.52, 2.0)), g=float(rng.uniform(-1e-3, 1e-3)), seed=300 + i))
    return cases


STUDY_CASES = draw_study_cases(24)


@pytest.mark.parametrize("case", STUDY_CASES, ids=[f"{i}" for i in range(len(STUDY_CASES))])
def test_random_layout_study_case_matches_oracle(case):
    """propagate bitwise and collide <= 1e-13 (relative to the weights)
    against the oracle, periodic in x and y."""
    from paper_1703_04594_amd import lbm
    c = case
    say(f"random study case {c}")
    lx, ly = c["lx"], c["ly"]
    f0 = WC * (1.0 + 0.02 * inputs.population_noise(lx, ly, c["seed"]))
    buf = lbm.study_pack(c["layout"], c["vl"], torch.tensor(f0, device=DEV))
    dst = torch.empty_like(buf)
    lbm.study_propagate(c["layout"], c["vl"], lx, ly, buf, dst)
    lbm.study_collide(c["layout"], c["vl"], lx, ly, c["tau"], c["g"], dst)
    got = lbm.study_unpack(c["layout"], c["vl"], lx, ly, dst).cpu().numpy()
    ref = oracle.RefLattice(lx, ly, c["tau"], c["g"], ybc=oracle.PERIODIC)
    ref.set_pops(f0)
    ref.propagate()
    ref.collide()
    err = float(np.max(np.abs(got - ref.get_pops()) / WC))
    assert err <= 1e-13, (c, err)


def draw_hetero_cases(n, seed=20170315):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(n):
        lx = int(rng.integers(9, 120))
        mmax = (lx - 3) // 2
        m = 0 if rng.random() < 0.15 else int(rng.integers(2, mmax + 1))
        cases.append(dict(lx=lx, ly=int(rng.integers(7, 200)), m=m, tau=float(rng.uniform(0.52, 2.0)),
                          g=float(rng.uniform(-1e-3, 1e-3)), tb=float(rng.uniform(0.7, 1.5)),
                          tt=float(rng.uniform(0.7, 1.5)), ybc=str(rng.choice(["walls", "periodic"])),
                          threads=int(rng.integers(1, 5)), n=int(rng.integers(1, 5)), seed=500 + i))
    return cases


HETERO_CASES = draw_hetero_cases(16)


@pytest.mark.parametrize("case", HETERO_CASES, ids=[f"{i}" for i in range(len(HETERO_CASES))])
def test_random_split_lattice_matches_oracle(case):
    from paper_1703_04594_amd.lbm import Hetero
    c = case
    say(f"random hetero case {c}")
    lx, ly = c["lx"], c["ly"]
    f0 = WC * (1.0 + 0.02 * inputs.population_noise(lx, ly, c["seed"]))
    h = Hetero(lx, ly, c["tau"], c["g"], c["tb"], c["tt"], ybc=c["ybc"], m=c["m"], host_threads=c["threads"],
               device=DEV)
    h.set_pops(f0)
    h.step(c["n"])
    got = h.get_pops()
    h.close()
    ref = oracle.RefLattice(lx, ly, c["tau"], c["g"], c["tb"], c["tt"],
                            ybc=oracle.WALL if c["ybc"] == "walls" else oracle.PERIODIC)
    ref.set_pops(f0)
    ref.step(c["n"])
    err = float(np.max(np.abs(got - ref.get_pops()) / WC))
    assert err <= 1e-12, (c, err)
