"""Gradients of a final-time objective with respect to the diffusion field D(x).

``simulate(D, spec)`` runs the TRT-R step `spec.nsteps` times on the GPU and returns phi at the final
time; it is a ``torch.autograd.Function`` whose backward pass runs the hand-written adjoint kernels
(``lbm_adjoint_step``: the transpose of the step's population Jacobian and the D-gradient, node by
node) in reverse.  The forward pass keeps a checkpoint every K = ceil(sqrt(T)) steps; the backward
pass reloads each checkpoint, recomputes the K states of its segment and walks them backwards, so
memory holds about 2 sqrt(T) states instead of T.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import torch

from . import lbm as L
from .solver import Solver


@dataclass
class RunSpec:
    """Everything but D that defines one periodic run (device FP64 fields [ny, nx])."""
    nx: int
    ny: int
    dx: float
    dt: float
    lam: float
    phi0: torch.Tensor
    ux: torch.Tensor
    uy: torch.Tensor
    nsteps: int
    mode: str = "f32"
    aux: int = L.LBM_AUX_LOCAL
    segment: Optional[int] = None          # checkpoint interval (default ceil(sqrt(nsteps)))
    stats: dict = field(default_factory=dict)


class _TRTRRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D: torch.Tensor, spec: RunSpec):
        p = L.make_params(spec.nx, spec.ny, spec.dx, spec.dt, spec.lam, float(D.mean()), spec.mode, spec.aux)
        fields = {"phi0": spec.phi0, "ux": spec.ux, "uy": spec.uy, "D": D.detach().to(torch.float64).contiguous()}
        solver = Solver([(p, fields)])
        T = int(spec.nsteps)
        K = int(spec.segment or max(1, math.ceil(math.sqrt(T))))
        ckpts = []
        t = 0
        while t < T:
            ckpts.append((t, solver.state_save()))
            n = min(K, T - t)
            solver.step(n)
            t += n
        _, phi = solver.macros(want_phi=True)
        ctx.solver, ctx.ckpts, ctx.T, ctx.K, ctx.spec = solver, ckpts, T, K, spec
        spec.stats.update(checkpoints=len(ckpts), segment=K)
        return phi

    @staticmethod
    def backward(ctx, dphi: torch.Tensor):
        solver, spec, T, K = ctx.solver, ctx.spec, ctx.T, ctx.K
        mdtype = torch.float64 if spec.mode == "f64" else torch.float32
        nbytes = L.lbm_adjoint_bytes(solver.ctx)
        lam_a = torch.empty(nbytes // mdtype.itemsize, dtype=mdtype, device="cuda")
        lam_b = torch.empty_like(lam_a)
        L.lbm_adjoint_seed(solver.ctx, 0, dphi.detach().to(torch.float64).contiguous(), lam_a)
        grad = torch.zeros((spec.ny, spec.nx), dtype=torch.float64, device="cuda")
        for t0, ck in reversed(ctx.ckpts):
            n = min(K, T - t0)
            solver.state_load(ck, t0)
            states = [solver.state_save()]
            for _ in range(n - 1):  # recompute the segment's states g^{t0} .. g^{t0+n-1}
                solver.step(1)
                states.append(solver.state_save())
            for j in reversed(range(n)):  # dL/dg^{t0+j} from dL/dg^{t0+j+1}
                L.lbm_adjoint_step(solver.ctx, 0, states[j], lam_a, lam_b, grad)
                lam_a, lam_b = lam_b, lam_a
        if spec.stats is not None:
            dphi0 = torch.empty((spec.ny, spec.nx), dtype=torch.float64, device="cuda")
            L.lbm_adjoint_init(solver.ctx, 0, lam_a, dphi0)
            spec.stats["dL_dphi0"] = dphi0
        solver.close()
        ctx.solver = None
        return grad, None


def simulate(D: torch.Tensor, spec: RunSpec) -> torch.Tensor:
    """phi at step spec.nsteps for the diffusion field D (device [ny, nx]); differentiable in D."""
    return _TRTRRun.apply(D, spec)


def bspline_operator(n_nodes: int, n_ctrl: int, device="cuda") -> torch.Tensor:
    """Periodic uniform cubic B-spline basis matrix [n_nodes, n_ctrl] (FP64): entry (j, a) is the cubic
    B-spline b3(t) at t = j n_ctrl / n_nodes - a, wrapped to the period n_ctrl, with
    b3(t) = (4 - 6|t|^2 + 3|t|^3)/6 for |t| < 1, (2 - |t|)^3/6 for 1 <= |t| < 2, else 0.  Every row
    is a partition of unity with positive weights, so a positive theta gives a positive D."""
    t = (torch.arange(n_nodes, dtype=torch.float64, device=device)[:, None] * (n_ctrl / n_nodes)
         - torch.arange(n_ctrl, dtype=torch.float64, device=device)[None, :])
    t = torch.remainder(t + n_ctrl / 2.0, float(n_ctrl)) - n_ctrl / 2.0
    a = t.abs()
    near = (4.0 - 6.0 * a * a + 3.0 * a ** 3) / 6.0
    far = torch.clamp(2.0 - a, min=0.0) ** 3 / 6.0
    return torch.where(a < 1.0, near, far)


def D_from_control(theta: torch.Tensor, By: torch.Tensor, Bx: torch.Tensor) -> torch.Tensor:
    """D = By theta Bx^T (bicubic B-spline surface), differentiable in theta."""
    return By @ theta @ Bx.transpose(0, 1)
