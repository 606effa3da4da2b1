"""PyTorch CPU float64 restatement of the oracle step, for exact gradients.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The gradient of a rollout is a plain definition -- the derivative of the
forward map -- so the reference gradient is that map written with PyTorch
operations (float64, CPU) and differentiated by autograd.  It restates the
same readings as ``lbm_ref.c`` (arXiv:1703.04594 section 3: eq. (1) BGK
update, eq. (2) moments, eq. (4) pull streaming; wall rule, gravity shift and
Hermite equilibrium as documented there) and takes the constants from the C
oracle.  A test ties this forward to the C oracle and pins autograd against
central finite differences of the C oracle.
"""
from __future__ import annotations

import numpy as np
import torch

from . import scale_c, velocity_table, weights

DT = torch.float64


class TorchD2Q37:
    def __init__(self, lx: int, ly: int, g_y: float = 0.0, t_bottom: float = 1.0,
                 t_top: float = 1.0, walls: bool = True):
        ex, ey = velocity_table()
        self.ex = [int(v) for v in ex]
        self.ey = [int(v) for v in ey]
        c = scale_c()
        self.w = torch.tensor(weights(), dtype=DT)
        self.xi_x = torch.tensor(c * ex.astype(np.float64), dtype=DT)
        self.xi_y = torch.tensor(c * ey.astype(np.float64), dtype=DT)
        self.lx, self.ly, self.g_y, self.walls = lx, ly, g_y, walls
        one = torch.ones((), dtype=DT)
        zero = torch.zeros((), dtype=DT)
        self.ew_bot = self.feq(one, zero, zero, torch.tensor(t_bottom, dtype=DT))
        self.ew_top = self.feq(one, zero, zero, torch.tensor(t_top, dtype=DT))

    # -- eq. (2) moments --------------------------------------------------
    def moments(self, f):
        xx = self.xi_x[:, None, None]
        yy = self.xi_y[:, None, None]
        rho = f.sum(0)
        ux = (xx * f).sum(0) / rho
        uy = (yy * f).sum(0) / rho
        e = (((xx - ux) ** 2 + (yy - uy) ** 2) * f).sum(0)
        return rho, ux, uy, e / (2.0 * rho)

    # -- 4th-order Hermite equilibrium, expanded form -----------------------
    def feq(self, rho, ux, uy, T):
        shape = torch.broadcast_shapes(rho.shape, ux.shape, uy.shape, T.shape)
        idx = (slice(None),) + (None,) * len(shape)
        xx, yy, w = self.xi_x[idx], self.xi_y[idx], self.w[idx]
        a = xx * ux + yy * uy
        u2 = ux * ux + uy * uy
        th = T - 1.0
        x2 = xx * xx + yy * yy
        h2 = (a * a - u2 + th * (x2 - 2.0)) / 2.0
        h3 = a * (a * a - 3.0 * u2 + 3.0 * th * (x2 - 4.0)) / 6.0
        h4 = (a ** 4 - 6.0 * a * a * u2 + 3.0 * u2 * u2
              + 6.0 * th * (a * a * (x2 - 6.0) + u2 * (4.0 - x2))
              + 3.0 * th * th * (x2 * x2 - 8.0 * x2 + 8.0)) / 24.0
        return w * rho * (1.0 + a + h2 + h3 + h4)

    # -- pull streaming and wall rule ---------------------------------------
    def stream(self, f):
        ly = self.ly
        rho = f.sum(0)
        out = []
        for l in range(37):
            ex, ey = self.ex[l], self.ey[l]
            p = torch.roll(f[l], shifts=(ex, ey), dims=(0, 1))
            if self.walls and ey != 0:
                rs = torch.roll(rho, shifts=ex, dims=0)          # rho(x - ex, .)
                if ey > 0:   # rows y < ey pull from below the bottom wall
                    ym = [ey - y - 1 for y in range(ey)]
                    p = torch.cat([self.ew_bot[l] * rs[:, ym], p[:, ey:]], dim=1)
                else:        # rows y >= ly + ey pull from above the top wall
                    ym = [2 * ly - 1 - (y - ey) for y in range(ly + ey, ly)]
                    p = torch.cat([p[:, :ly + ey], self.ew_top[l] * rs[:, ym]], dim=1)
            out.append(p)
        return torch.stack(out)

    # -- eq. (1) BGK relaxation with the gravity shift -----------------------
    def collide(self, g, tau):
        rho, ux, uy, T = self.moments(g)
        uys = uy + tau * self.g_y
        Ts = T + tau * (1.0 - tau) * self.g_y ** 2 / 2.0
        feq = self.feq(rho, ux, uys, Ts)
        return g - (g - feq) / tau

    def step(self, f, tau):
        return self.collide(self.stream(f), tau)

    # -- Rayleigh-Taylor initial state from the interface displacement P ----
    def rt_fields(self, P, t_mid=1.0, t_amp=1.0 / 3.0, p0=8.0 / 9.0, width=2.0, y_mid=None):
        if y_mid is None:
            y_mid = (self.ly - 1) / 2.0
        y = torch.arange(self.ly, dtype=DT)[None, :]
        T0 = t_mid - t_amp * torch.tanh((y - y_mid - P) / width)
        return p0 / T0, T0

    def init_rt(self, P, **kw):
        rho0, T0 = self.rt_fields(P, **kw)
        z = torch.zeros_like(T0)
        return self.feq(rho0, z, z, T0)

    def temperature(self, f):
        return self.moments(f)[3]

    def rollout_T(self, P, tau, nsteps, **kw):
        f = self.init_rt(P, **kw)
        for _ in range(nsteps):
            f = self.step(f, tau)
        return self.temperature(f)
