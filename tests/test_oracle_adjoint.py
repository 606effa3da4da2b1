"""Pins of the gradient oracle (CPU only).

The torch restatement must reproduce the C oracle's forward, and its autograd
gradients must match central finite differences of the C oracle's forward:
the derivative of the forward map is the definition the adjoint must meet.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.ref_torch import TorchD2Q37
from paper_1703_04594_amd import inputs

TB, TT, G, TAU = 4 / 3, 2 / 3, -1e-5, 0.7


def c_oracle_T(P, tau, n, lx, ly, g=G):
    y = np.arange(ly)[None, :]
    T0 = 1.0 - np.tanh((y - (ly - 1) / 2 - P) / 2.0) / 3.0
    L = oracle.RefLattice(lx, ly, tau, g, TB, TT)
    L.init((8 / 9) / T0, 0.0, 0.0, T0)
    L.step(n)
    return L.macros()[3]


def test_torch_forward_matches_c_oracle():
    lx, ly, n = 24, 20, 12
    P = inputs.rt_perturbation(lx, ly, 3)
    m = TorchD2Q37(lx, ly, G, TB, TT)
    with torch.no_grad():
        T = m.rollout_T(torch.tensor(P), TAU, n).numpy()
    Tc = c_oracle_T(P, TAU, n, lx, ly)
    assert np.max(np.abs(T - Tc)) <= 1e-13


def test_torch_forward_matches_c_oracle_periodic_populations():
    lx, ly = 10, 9
    w = oracle.weights()
    f0 = w[:, None, None] * (1 + 0.05 * inputs.population_noise(lx, ly, 4))
    L = oracle.RefLattice(lx, ly, TAU, 1e-3, ybc=oracle.PERIODIC)
    L.set_pops(f0)
    L.step(3)
    m = TorchD2Q37(lx, ly, 1e-3, walls=False)
    f = torch.tensor(f0)
    with torch.no_grad():
        for _ in range(3):
            f = m.step(f, TAU)
    assert np.max(np.abs(f.numpy() - L.get_pops()) / w[:, None, None]) <= 1e-13


@pytest.mark.parametrize("g", [G, -2e-3])
def test_autograd_matches_central_differences_of_c_oracle(g):
    lx, ly, n = 12, 14, 10
    P = inputs.rt_perturbation(lx, ly, 5) + 1e-3 * inputs.uniform_field(lx, ly, 6, -1, 1)
    Tstar = c_oracle_T(inputs.rt_perturbation(lx, ly, 9), TAU, n, lx, ly, g)
    m = TorchD2Q37(lx, ly, g, TB, TT)
    Pt = torch.tensor(P, requires_grad=True)
    tau_t = torch.tensor(TAU, dtype=torch.float64, requires_grad=True)
    T = m.rollout_T(Pt, tau_t, n)
    loss = 0.5 * ((T - torch.tensor(Tstar)) ** 2).sum()
    loss.backward()
    gP, gtau = Pt.grad.numpy(), float(tau_t.grad.detach())

    def L(Pv, tau):
        return 0.5 * np.sum((c_oracle_T(Pv, tau, n, lx, ly, g) - Tstar) ** 2)

    eps = 1e-4
    for v in inputs.probe_directions(lx, ly, 21, 3):
        fd = (L(P + eps * v, TAU) - L(P - eps * v, TAU)) / (2 * eps)
        ad = float(np.sum(gP * v))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    # the loss is strongly curved in tau on a lattice this small: at eps = 1e-4
    # the central difference still carries ~3e-4 truncation error, at 1e-6 it
    # agrees with autograd to ~4e-8
    eps = 1e-6
    fd = (L(P, TAU + eps) - L(P, TAU - eps)) / (2 * eps)
    assert abs(fd - gtau) <= 1e-6 * abs(gtau), (fd, gtau)
