"""Host + GPU co-execution: the performance model of section 6 and its
auto-tuning (host-side logic; the stepping itself is lbm.Hetero, native).

The lattice is split along x: m border columns on each side run on the
host's cores, the other lx - 2m on the GPU, and three-column halos are
swapped after every step.  The model (eq. (perf-model), one process, so no
inter-process term) is

    T_exe(m) = max(T_acc, T_host) + T_swap
    T_acc    = (lx - 2m) ly tau_d
    T_host   = 2m ly tau_h

with T_swap independent of m (and absent when m = 0: nothing is split).
T_exe is least where T_acc = T_host (eq. (param-tuning)):
2m* = lx tau_d / (tau_d + tau_h).  The auto-tuner measures tau_d, tau_h and
T_swap with short runs and evaluates the model.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Model:
    tau_d: float     # GPU seconds per site and step
    tau_h: float     # host seconds per site and step
    t_swap: float    # halo swap seconds per step

    def t_exe(self, lx: int, ly: int, m: int) -> float:
        if m == 0:
            return lx * ly * self.tau_d
        return max((lx - 2 * m) * ly * self.tau_d, 2 * m * ly * self.tau_h) + self.t_swap

    def mlups(self, lx: int, ly: int, m: int) -> float:
        return lx * ly / self.t_exe(lx, ly, m) / 1e6

    def m_balance(self, lx: int) -> float:
        """The real m at which T_acc = T_host."""
        return 0.5 * lx * self.tau_d / (self.tau_d + self.tau_h)

    def best_m(self, lx: int, ly: int) -> int:
        """The admissible m (0, or 2 <= m with lx - 2m >= 3) of least
        predicted T_exe; the balance point's neighbours and 0 are the only
        candidates, since T_exe falls up to the balance and rises after it."""
        mb = self.m_balance(lx)
        cands = {0} | {m for m in (int(np.floor(mb)), int(np.ceil(mb))) if m >= 2 and lx - 2 * m >= 3}
        if mb < 2 and lx - 4 >= 3:
            cands.add(2)
        return min(sorted(cands), key=lambda m: self.t_exe(lx, ly, m))


def autotune(make, lx: int, ly: int, m_probe: int, steps: int = 20, warmup: int = 3) -> Model:
    """Mini-benchmarks on the lattice itself: `make(m)` returns a ready
    lbm.Hetero with m border columns per side.  tau_d from the GPU alone
    (m = 0), tau_h and T_swap from a split run with m_probe columns."""
    h = make(0)
    h.step(warmup)
    h.step(steps)
    tau_d = h.times()["gpu"] / (lx * ly)
    h.close()
    h = make(m_probe)
    h.step(warmup)
    h.step(steps)
    t = h.times()
    h.close()
    return Model(tau_d=tau_d, tau_h=t["host"] / (2 * m_probe * ly), t_swap=t["swap"])
