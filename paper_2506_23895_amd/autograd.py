"""torch.autograd.Function around the C ABI: J(gamma) forward, dJ/dgamma backward.

forward() runs lks_forward on the device tensor gamma (Algorithm 1 with state checkpoints);
backward() runs lks_adjoint (restore each checkpoint, recompute its segment, exact reverse
steps and the atomic-free sensitivity gather) and lks_sensitivity, then scales by the incoming
gradient.  torch supplies only the tensors and the stream.
"""
from __future__ import annotations

import torch

from . import lks


class Evaluator:
    """Owns one device-IO context for a workload; hands out J(gamma) as an autograd node."""

    def __init__(self, cfg: dict, hbm_budget: int = 0):
        self.cfg = cfg
        self.dtype = torch.float64 if cfg["precision"] == "F64" else torch.float32
        stream = torch.cuda.current_stream().cuda_stream
        self.solver = lks.Solver(cfg, io_on_device=True, stream=stream, hbm_budget=hbm_budget)
        self.generation = 0   # bumps on every forward; backward checks it still matches

    def __call__(self, gamma: torch.Tensor) -> torch.Tensor:
        return LKSFunction.apply(gamma, self)

    def close(self) -> None:
        self.solver.close()


class LKSFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma: torch.Tensor, ev: Evaluator) -> torch.Tensor:
        if not gamma.is_cuda or gamma.dtype != ev.dtype:
            raise TypeError(f"gamma must be a CUDA tensor of dtype {ev.dtype}")
        g = gamma.detach().contiguous()
        J = ev.solver.forward(g)
        ev.generation += 1
        ctx.ev = ev
        ctx.gen = ev.generation
        ctx.save_for_backward(g)
        return torch.tensor(J, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        ev = ctx.ev
        (g,) = ctx.saved_tensors
        if ev.generation != ctx.gen:  # another forward ran since: rebuild this trajectory
            ev.solver.forward(g)
            ev.generation += 1
        ev.solver.adjoint()
        out = torch.empty_like(g)
        ev.solver.sensitivity(out)
        return (gJ.to(out.dtype) * out), None
