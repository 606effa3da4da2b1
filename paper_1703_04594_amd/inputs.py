"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

This module only draws random numbers and lays them out; it holds none of the
lattice Boltzmann arithmetic, so the GPU path and the CPU oracle can both be
fed from it without sharing any of the method's code.

Recipes (all FP64, numpy ``default_rng`` streams keyed by an integer seed):

* ``rt_perturbation`` -- the interface displacement field P(x, y) of the
  Rayleigh-Taylor set-up: one uniform draw in [-1, 1) per lattice column,
  scaled by the amplitude (1e-3 lattice units) and repeated along y.
* ``population_noise`` -- standard normal numbers in the canonical population
  layout [37][lx][ly], used to build non-equilibrium test states.
* ``probe_directions`` -- k standard normal fields of shape (lx, ly) for
  directional finite-difference checks, scaled to unit 2-norm ("l2") or to
  unit root-mean-square per site ("rms").
* ``uniform_field`` -- uniform numbers in [lo, hi) of shape (lx, ly).
"""
from __future__ import annotations

import numpy as np

NPOP = 37


def rt_perturbation(lx: int, ly: int, seed: int, amplitude: float = 1e-3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    eta = rng.uniform(-1.0, 1.0, size=(lx, 1))
    return np.ascontiguousarray(np.broadcast_to(amplitude * eta, (lx, ly)), dtype=np.float64)


def population_noise(lx: int, ly: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((NPOP, lx, ly))


def probe_directions(lx: int, ly: int, seed: int, k: int, norm: str = "l2") -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((k, lx, ly))
    v /= np.sqrt((v * v).sum(axis=(1, 2), keepdims=True))
    if norm == "rms":
        v *= np.sqrt(lx * ly)
    return v


def uniform_field(lx: int, ly: int, seed: int, lo: float, hi: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(lx, ly))
