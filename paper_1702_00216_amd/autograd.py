"""torch.autograd.Function around the TCM forward and its adjoint.

Forward: receiver traces of a single-shot TCM run with wave speed ``c``.
Backward: dL/dc from dL/dtraces through ``tcm_adjoint`` (time-reversed
adjoint field with checkpoint-and-recompute of the forward, all on the GPU).
Only argument marshalling happens here.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

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


class TCMForward(torch.autograd.Function):
    """traces = TCMForward.apply(c, spec); c is a (nz, ny, nx) float32 tensor."""

    @staticmethod
    def forward(ctx, c: torch.Tensor, spec: ShotSpec):
        nz, ny, nx = c.shape
        c_host = np.ascontiguousarray(c.detach().to("cpu", torch.float32).numpy())
        sim = Simulation((nx, ny, nz), spec.dx, spec.dt, c_host, spec.trigger, spec.retire,
                         pool_bytes=spec.pool_bytes, checkpoint_every=spec.checkpoint_every)
        sim.add_source(spec.source, spec.wavelet)
        sim.set_receivers(spec.receivers)
        sim.step(spec.nt)
        traces = torch.from_numpy(sim.read_traces()).to(c.device)
        ctx.sim = sim
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
        sim.close()
        ctx.sim = None
        return out.to(ctx.c_device), None


def tcm_traces(c: torch.Tensor, spec: ShotSpec) -> torch.Tensor:
    return TCMForward.apply(c, spec)
