"""Host + GPU co-execution: the performance model of section 6 and its
auto-tuning (host-side logic; the stepping itself is lbm.Hetero, native).

The lattice is split along x: m border columns on each side run on the
host's cores, the other lx - 2m on the GPU, and three-column halos are
swapped after every step.  The performance model of section 6 (one process,
so no inter-process term) is

    T_exe(m) = max(T_acc, T_host) + T_swap
    T_acc    = (lx - 2m) ly tau_d
    T_host   = 2m ly tau_h

with T_swap independent of m (and absent when m = 0: nothing is split).
T_exe is least where T_acc = T_host (the tuning condition of section 6):
2m* = lx tau_d / (tau_d + tau_h).  The auto-tuner measures tau_d, tau_h and
T_swap with short runs and evaluates the model.

A single tau_h, measured at one band width, does not hold across widths on a
many-core host: the band (2m columns plus 3 halo columns per side) is split
over the threads by whole columns, so narrow bands leave threads idle, and a
wide band's working set outgrows the caches.  The model therefore also takes
T_host(m) measured per width by host-only runs of the same band
(`host_times`), interpolated linearly in m between measured widths; tau_h
then is T_host(m) / (2m ly).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Model:
    tau_d: float     # GPU seconds per site and step
    tau_h: float     # host seconds per site and step (one width)
    t_swap: float    # halo swap seconds per step
    host_times: dict | None = None   # m -> host step seconds (host-only runs)

    def t_host(self, ly: int, m: int) -> float:
        """Host step time of a band of m columns per side."""
        if not self.host_times:
            return 2 * m * ly * self.tau_h
        ms = sorted(self.host_times)
        if m <= ms[0]:                 # beyond the measured widths: nearest width's rate per site
            return self.host_times[ms[0]] * m / ms[0]
        if m >= ms[-1]:
            return self.host_times[ms[-1]] * m / ms[-1]
        return float(np.interp(m, ms, [self.host_times[k] for k in ms]))

    def t_exe(self, lx: int, ly: int, m: int) -> float:
        if m == 0:
            return lx * ly * self.tau_d
        return max((lx - 2 * m) * ly * self.tau_d, self.t_host(ly, m)) + self.t_swap

    def mlups(self, lx: int, ly: int, m: int) -> float:
        return lx * ly / self.t_exe(lx, ly, m) / 1e6

    def m_balance(self, lx: int) -> float:
        """The real m at which T_acc = T_host."""
        return 0.5 * lx * self.tau_d / (self.tau_d + self.tau_h)

    def best_m(self, lx: int, ly: int) -> int:
        """The admissible m (0, or 2 <= m with lx - 2m >= 3) of least
        predicted T_exe.  With one tau_h the balance point's neighbours and
        0 are the only candidates, since T_exe falls up to the balance and
        rises after it; with measured host times every admissible m is
        evaluated."""
        if self.host_times:
            cands = [0] + list(range(2, (lx - 3) // 2 + 1))
            return min(cands, key=lambda m: self.t_exe(lx, ly, m))
        mb = self.m_balance(lx)
        cands = {0} | {m for m in (int(np.floor(mb)), int(np.ceil(mb))) if m >= 2 and lx - 2 * m >= 3}
        if mb < 2 and lx - 4 >= 3:
            cands.add(2)
        return min(sorted(cands), key=lambda m: self.t_exe(lx, ly, m))


def autotune(make, lx: int, ly: int, m_probe: int, steps: int = 20, warmup: int = 10, repeats: int = 3,
             host_probe=None, host_widths=()) -> Model:
    """Mini-benchmarks on the lattice itself: `make(m)` returns a ready
    lbm.Hetero with m border columns per side.  tau_d from the GPU alone
    (m = 0), tau_h and T_swap from a split run with m_probe columns; each the
    median of `repeats` runs of `steps` steps after `warmup` steps (a single
    short run's exchange time has come out several times too long).  With
    `host_probe(m)` (host step seconds of an m-column band, run on the host
    alone), T_host is also measured at every width in `host_widths`."""
    def timed(m):
        h = make(m)
        h.step(warmup)
        runs = []
        for _ in range(repeats):
            h.step(steps)
            runs.append(h.times())
        h.close()
        return {k: float(np.median([r[k] for r in runs])) for k in runs[0]}
    tau_d = timed(0)["gpu"] / (lx * ly)
    t = timed(m_probe)
    host_times = {int(m): float(host_probe(m)) for m in host_widths} if host_probe else None
    return Model(tau_d=tau_d, tau_h=t["host"] / (2 * m_probe * ly), t_swap=t["swap"], host_times=host_times)
