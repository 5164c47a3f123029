"""torch.autograd.Function around the TCM forward and its adjoint.

Forward: receiver traces of a single-shot TCM run with wave speed ``c``.
Backward: dL/dc from dL/dtraces through ``tcm_adjoint`` (time-reversed
adjoint field with checkpoint-and-recompute of the forward, all on the GPU).
Only argument marshalling happens here.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from .sim import Simulation


@dataclass
class ShotSpec:
    """Everything about one shot except the wave speed."""
    dx: float
    dt: float
    source: Sequence[int]            # (x, y, z)
    wavelet: np.ndarray              # float32 samples
    receivers: np.ndarray            # (nrec, 3) int
    nt: int                          # steps (= recorded trace rows)
    checkpoint_every: int = 50
    trigger: float = 0.0
    retire: float = 0.0
    pool_bytes: int = 0


# Idle handles by geometry and configuration.  A forward takes one (giving
# it the new wave speed with tcm_set_media, which keeps its allocations) or
# makes one; the backward hands it back, so an inversion loop creates a
# handle once per concurrently live forward, not once per iteration.
_IDLE: Dict[tuple, List[Simulation]] = {}


def _config_key(shape, spec: ShotSpec) -> tuple:
    return (tuple(shape), float(spec.dx), float(spec.dt), float(spec.trigger), float(spec.retire),
            int(spec.pool_bytes), int(spec.checkpoint_every))


def release_handles() -> None:
    """Destroy the idle handles kept for reuse."""
    for sims in _IDLE.values():
        for s in sims:
            s.close()
    _IDLE.clear()


class TCMForward(torch.autograd.Function):
    """traces = TCMForward.apply(c, spec); c is a (nz, ny, nx) float32 tensor."""

    @staticmethod
    def forward(ctx, c: torch.Tensor, spec: ShotSpec):
        nz, ny, nx = c.shape
        c_host = np.ascontiguousarray(c.detach().to("cpu", torch.float32).numpy())
        key = _config_key((nx, ny, nz), spec)
        idle = _IDLE.get(key)
        if idle:
            sim = idle.pop()
            sim.set_media(c_host)
        else:
            sim = Simulation((nx, ny, nz), spec.dx, spec.dt, c_host, spec.trigger, spec.retire,
                             pool_bytes=spec.pool_bytes, checkpoint_every=spec.checkpoint_every)
        sim.add_source(spec.source, spec.wavelet)
        sim.set_receivers(spec.receivers)
        sim.step(spec.nt)
        traces = torch.from_numpy(sim.read_traces()).to(c.device)
        ctx.sim = sim
        ctx.key = key
        ctx.c_device = c.device
        return traces

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        sim: Optional[Simulation] = ctx.sim
        g = grad_traces.detach().to(torch.float32).contiguous()
        if g.is_cuda:
            out = torch.empty(tuple(reversed(sim.shape)), dtype=torch.float32, device=g.device)
            sim.adjoint_device(g, out)
        else:
            out = torch.from_numpy(sim.adjoint(g.numpy()))
        _IDLE.setdefault(ctx.key, []).append(sim)
        ctx.sim = None
        return out.to(ctx.c_device), None


def tcm_traces(c: torch.Tensor, spec: ShotSpec) -> torch.Tensor:
    return TCMForward.apply(c, spec)
