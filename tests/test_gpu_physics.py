"""Closed-form physics on the GPU path itself, in every storage precision
(an independent check of the FP32 forms, beside their parity with the FP64
oracle): a small shear wave decays as exp(-nu k^2 t) with
nu = T (tau - 1/2) / c^2 (section 3's continuum limit, lattice units), and
steady conduction between two walls gives a linear, x-uniform temperature
profile."""
import numpy as np
import pytest
import torch

from paper_1703_04594_amd import lbm
from paper_1703_04594_amd.lbm import Lattice

from _util import say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PRECISIONS = ["fp64", "fp32", "fp32_f32sums"]


def field(v, lx, ly):
    return torch.as_tensor(np.broadcast_to(v, (lx, ly)).copy(), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("step", ["fused", "split"])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_shear_wave_decays_at_the_viscous_rate(precision, step):
    lx, ly, tau, U, T0 = 16, 128, 0.7, 1e-4, 1.0
    say(f"shear wave {precision} {step}")
    y = np.arange(ly)
    s = np.sin(2 * np.pi * y / ly)
    lat = Lattice(lx, ly, tau, precision=precision, ybc="periodic", step=step, device=DEV)
    lat.init(field(1.0, lx, ly), field(U * s[None, :], lx, ly), field(0.0, lx, ly), field(T0, lx, ly))
    amps, t = {}, 0
    for mark in (200, 2000):
        lat.step(mark - t)
        t = mark
        ux = lat.macros()[1].cpu().numpy()
        amps[mark] = 2.0 / ly * float(np.sum(ux.mean(axis=0) * s))
    rate = np.log(amps[200] / amps[2000]) / 1800.0
    nu = T0 * (tau - 0.5) / lbm.scale_c() ** 2
    k = 2 * np.pi / ly
    say(f"  rate / (nu k^2) = {rate / (nu * k * k):.5f}")
    assert abs(rate / (nu * k * k) - 1.0) < 0.01, (rate, nu * k * k)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_conduction_between_walls_is_linear(precision):
    lx, ly, tau, tb, tt = 8, 24, 0.7, 1.05, 0.95
    say(f"conduction {precision}")
    lat = Lattice(lx, ly, tau, 0.0, tb, tt, precision=precision, step="fused", device=DEV)
    lat.init(field(1.0, lx, ly), field(0.0, lx, ly), field(0.0, lx, ly), field(1.0, lx, ly))
    lat.step(20000)
    _, ux, uy, T = (t.cpu().numpy() for t in lat.macros())
    prof = T.mean(axis=0)
    yy = np.arange(ly)
    A = np.vstack([yy, np.ones(ly)]).T
    coef, res, *_ = np.linalg.lstsq(A, prof, rcond=None)
    r2 = 1.0 - res[0] / np.sum((prof - prof.mean()) ** 2)
    say(f"  R^2 = {r2:.6f}, slope {coef[0]:.3e}")
    assert r2 > 0.999, r2
    assert coef[0] < 0 and prof[0] < tb and prof[-1] > tt
    # x-uniform to the storage precision's rounding
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert np.max(np.abs(T - prof[None, :])) < tol
    assert np.max(np.abs(ux)) < tol
    assert np.max(np.abs(uy)) < 5e-3
