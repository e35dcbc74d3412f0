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
    """Everything but D that defines one periodic run (device FP64 fields [ny, nx]).

    The first forward pass creates one library context (with a D field) and keeps it in the spec;
    later passes replace D (``lbm_set_diffusion``) and restart from the stored initial state
    (``lbm_state_load``), so a gradient loop over D pays for ``lbm_init`` once.  ``close()`` releases
    the context."""
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
    _solver: Optional[Solver] = field(default=None, repr=False)
    _init_state: Optional[torch.Tensor] = field(default=None, repr=False)

    def solver_for(self, D: torch.Tensor) -> Solver:
        """The run's context with diffusion field D, reset to the initial state g_eq(phi0, u)."""
        D = D.detach().to(torch.float64).contiguous()
        if self._solver is None:
            p = L.make_params(self.nx, self.ny, self.dx, self.dt, self.lam, float(D.mean()), self.mode, self.aux)
            self._solver = Solver([(p, {"phi0": self.phi0, "ux": self.ux, "uy": self.uy, "D": D})])
            self._init_state = self._solver.state_save()
        else:
            self._solver.set_diffusion(D)
            self._solver.state_load(self._init_state, 0)
        return self._solver

    def close(self) -> None:
        if self._solver is not None:
            self._solver.close()
            self._solver = None
            self._init_state = None


class _TRTRRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D: torch.Tensor, spec: RunSpec):
        solver = spec.solver_for(D)
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
        ctx.ckpts, ctx.T, ctx.K, ctx.spec = ckpts, T, K, spec
        ctx.save_for_backward(D)
        spec.stats.update(checkpoints=len(ckpts), segment=K)
        return phi

    @staticmethod
    def backward(ctx, dphi: torch.Tensor):
        spec, T, K = ctx.spec, ctx.T, ctx.K
        (D,) = ctx.saved_tensors
        solver = spec.solver_for(D)  # the D of this forward pass, whatever ran in between
        mdtype = torch.float64 if spec.mode == "f64" else torch.float32
        nbytes = L.lbm_adjoint_bytes(solver.ctx)
        lam = torch.empty(nbytes // mdtype.itemsize, dtype=mdtype, device="cuda")
        lam_tmp = torch.empty_like(lam)
        sb = L.lbm_state_bytes(solver.ctx)
        states = torch.empty(K * sb, dtype=torch.uint8, device="cuda")
        grad = torch.zeros((spec.ny, spec.nx), dtype=torch.float64, device="cuda")
        with torch.cuda.stream(solver.stream):
            L.lbm_adjoint_seed(solver.ctx, 0, dphi.detach().to(torch.float64).contiguous(), lam)
            for t0, ck in reversed(ctx.ckpts):
                # each segment: its checkpoint into image 0, then recomputation and K adjoint steps,
                # enqueued by the library in one call
                states[:sb].copy_(ck)
                L.lbm_adjoint_segment(solver.ctx, 0, states, min(K, T - t0), lam, lam_tmp, grad)
            if spec.stats is not None:
                dphi0 = torch.empty((spec.ny, spec.nx), dtype=torch.float64, device="cuda")
                L.lbm_adjoint_init(solver.ctx, 0, lam, dphi0)
                spec.stats["dL_dphi0"] = dphi0
        ctx.ckpts = None
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
