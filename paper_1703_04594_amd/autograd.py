"""torch.autograd.Function over the GPU forward and hand-written adjoint.

``rt_temperature(P, tau, cfg)`` returns the temperature field T_N after
cfg.nsteps steps of the Rayleigh-Taylor run started from the interface
displacement field P.  Its backward seeds the adjoint with the incoming
dL/dT_N (lbm_adjoint_seed_temperature), reverses the N steps with the chosen
checkpoint schedule (lbm_adjoint_step per step, replaying forward segments
from stored states), and maps lambda_0 to dL/dP (lbm_adjoint_init_rt); the
d/dtau terms of every step are kept in per-block FP64 sums in the lattice and
added to one FP64 device scalar at the end of the sweep
(lbm_adjoint_take_dtau).

Forward states may be FP32-shifted (the adjoint then linearises around the
stored FP32 states, in FP64) or FP64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import checkpoint
from .lbm import Lattice, RtProfile


@dataclass
class RolloutConfig:
    lx: int
    ly: int
    nsteps: int
    g_y: float = -1e-5
    t_bottom: float = 4.0 / 3.0
    t_top: float = 2.0 / 3.0
    precision: str = "fp32"
    step: str = "fused"
    checkpoint: str = "sqrt"            # "sqrt" or "binomial"
    slots: int | None = None             # binomial: stored states
    memory_budget: int | None = None     # binomial: bytes for stored states (alternative to slots)
    lambda_precision: str = "fp64"      # adjoint state storage: "fp64" or "fp32"
    profile: RtProfile = field(default_factory=RtProfile)
    stats: dict = field(default_factory=dict)

    def schedule(self, state_bytes: int) -> checkpoint.Schedule:
        if self.checkpoint == "sqrt":
            return checkpoint.sqrt_schedule(self.nsteps)
        if self.checkpoint == "binomial":
            slots = self.slots
            if slots is None:
                if not self.memory_budget:
                    raise ValueError("binomial checkpointing needs slots or memory_budget")
                slots = max(1, self.memory_budget // state_bytes - 1)   # one working copy
            return checkpoint.binomial_schedule(self.nsteps, int(slots))
        raise ValueError(self.checkpoint)


class RTRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P: torch.Tensor, tau: torch.Tensor, cfg: RolloutConfig):
        lat = Lattice(cfg.lx, cfg.ly, float(tau), cfg.g_y, cfg.t_bottom, cfg.t_top,
                      precision=cfg.precision, step=cfg.step, adjoint=cfg.lambda_precision, device=P.device)
        P = P.detach().contiguous()
        lat.init_rt(P, cfg.profile)
        sch = cfg.schedule(lat.state_bytes)
        fwd, bwd = sch.split_at_first_adjoint()
        dacc = torch.zeros((), dtype=torch.float64, device=P.device)
        ex = checkpoint.Executor(lat, dacc)
        ex.run(fwd)
        ex.materialize()     # the lattice holds f_{N-1}
        lat.step(1)          # f_N
        T = lat.macros()[3]
        ctx.lat, ctx.ex, ctx.bwd, ctx.P, ctx.cfg = lat, ex, bwd, P, cfg
        cfg.stats.update(schedule_forward_steps=sch.forward_steps(), slots=sch.slots_needed,
                         state_bytes=lat.state_bytes)
        return T

    @staticmethod
    def backward(ctx, gT: torch.Tensor):
        lat, ex = ctx.lat, ctx.ex
        lat.seed_temperature(gT.detach().to(torch.float64).contiguous())
        ex.run(ctx.bwd)
        dP = lat.adjoint_init_rt(ctx.P, ctx.cfg.profile)
        dtau = ex.dtau.clone()
        ctx.cfg.stats.update(forward_steps=ex.forward_steps + 1, adjoint_steps=ex.adjoint_steps,
                             peak_slots=ex.peak_slots)
        ctx.lat = ctx.ex = None
        return dP, dtau, None


def rt_temperature(P: torch.Tensor, tau: torch.Tensor, cfg: RolloutConfig) -> torch.Tensor:
    return RTRollout.apply(P, tau, cfg)
