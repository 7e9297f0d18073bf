"""torch.autograd front end of the adjoint gradient (fdtd_grad_eps).

    problem = ProbeProblem(nx, ny, nz, dt, dx, dy, dz, eps_background, design_box,
                           nsteps, probe, source=Source(...))
    J = probe_energy(eps_design, problem)      # 0-dim float64 tensor
    J.backward()                               # eps_design.grad = dJ/d eps_r

J is the time-integrated |E|^2 at the probe node of the fundamental ADI run
(see fdtd_grad_eps in include/fdtd.h).  The forward call runs the library's
forward sweep; when a gradient is needed it also runs the checkpointed
adjoint sweep and keeps dJ/d eps_r for backward.  PyTorch only carries the
tensors: every step runs in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import Plan, Source


@dataclass
class ProbeProblem:
    nx: int
    ny: int
    nz: int
    dt: float
    dx: float
    dy: float
    dz: float
    eps_background: torch.Tensor          # (nz, ny, nx) eps_r outside the design cells
    design_box: tuple                     # (i0, i1, j0, j1, k0, k1), cells
    nsteps: int
    probe: tuple                          # node (i, j, k)
    source: Source | None = None
    E0: list | None = None                # initial fields (default zero)
    H0: list | None = None
    dtype: torch.dtype = torch.float32    # field storage
    solve_dtype: torch.dtype | None = None
    ckpt_every: int = 50
    device: torch.device | None = None

    def design_shape(self):
        i0, i1, j0, j1, k0, k1 = self.design_box
        return (k1 - k0, j1 - j0, i1 - i0)


def _eps_full(eps_design, pb: ProbeProblem):
    i0, i1, j0, j1, k0, k1 = pb.design_box
    eps = pb.eps_background.detach().to(device=eps_design.device, dtype=torch.float32).clone()
    eps[k0:k1, j0:j1, i0:i1] = eps_design.detach().to(torch.float32)
    return eps


def _fields(pb: ProbeProblem, device):
    shape = (pb.nz + 1, pb.ny + 1, pb.nx + 1)
    if pb.E0 is not None and pb.H0 is not None:
        return list(pb.E0), list(pb.H0)
    E = [torch.zeros(shape, dtype=pb.dtype, device=device) for _ in range(3)]
    H = [torch.zeros(shape, dtype=pb.dtype, device=device) for _ in range(3)]
    return E, H


class ProbeEnergy(torch.autograd.Function):
    """J(eps_design) with dJ/d eps_design from the adjoint of the fundamental ADI."""

    @staticmethod
    def forward(ctx, eps_design, pb: ProbeProblem):
        if tuple(eps_design.shape) != pb.design_shape():
            raise ValueError(f"eps_design must have shape {pb.design_shape()}")
        dev = pb.device if pb.device is not None else eps_design.device
        if dev.type != "cuda":
            raise ValueError("eps_design must live on the GPU (the library has no CPU path)")
        ctx.in_dtype = eps_design.dtype
        eps = _eps_full(eps_design.to(dev), pb)
        E, H = _fields(pb, dev)
        plan = Plan(pb.nx, pb.ny, pb.nz, pb.dt, pb.dx, pb.dy, pb.dz, scheme="adi", form="fundamental",
                    dtype=pb.dtype, eps_r=eps, device=dev, solve_dtype=pb.solve_dtype)
        try:
            if ctx.needs_input_grad[0]:
                J, g = plan.grad_eps(E, H, pb.nsteps, pb.probe, pb.source, pb.design_box, pb.ckpt_every)
                ctx.save_for_backward(g)
            else:
                J, _ = plan.grad_eps(E, H, pb.nsteps, pb.probe, pb.source)
        finally:
            plan.close()
        return torch.tensor(J, dtype=torch.float64, device=eps_design.device)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return (gJ.to(device=g.device, dtype=torch.float64) * g).to(ctx.in_dtype), None


def probe_energy(eps_design: torch.Tensor, pb: ProbeProblem) -> torch.Tensor:
    """J as a 0-dim float64 tensor, differentiable with respect to eps_design."""
    return ProbeEnergy.apply(eps_design, pb)
