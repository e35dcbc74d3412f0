"""Convenience wrapper over the C ABI: owns a torch workspace and one library context."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import lbm as L


class Solver:
    """One or more periodic instances advanced together on the current (or given) stream.

    instances: sequence of (params, fields) pairs; params from ``lbm.make_params``; fields a dict of
    device FP64 tensors ``phi0``, ``ux``, ``uy`` and optional ``D``, each [ny, nx].
    """

    def __init__(self, instances: Sequence, stream: Optional[torch.cuda.Stream] = None):
        self.params = [p for p, _ in instances]
        self.stream = stream or torch.cuda.current_stream()
        nbytes = L.lbm_workspace_size(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.ctx = L.lbm_init(self.params, [f for _, f in instances], self.workspace, self.stream)
        self._keep = None

    def step(self, nsteps: int, ux=None, uy=None, S=None, dSdt=None) -> None:
        self._keep = (ux, uy, S, dSdt)  # inputs stay alive until the next call
        L.lbm_step(self.ctx, nsteps, ux, uy, S, dSdt)

    def _shape(self, inst: int):
        p = self.params[inst]
        return (p.ny, p.nx) if p.lattice == L.LBM_LATTICE_D2Q9 else (p.nz, p.ny, p.nx)

    def _q(self, inst: int) -> int:
        return L.LATTICE_Q[self.params[inst].lattice]

    def set_velocity(self, ux: torch.Tensor, uy: torch.Tensor, uz: Optional[torch.Tensor] = None,
                     inst: int = 0) -> None:
        self._keep_u = (ux, uy, uz)
        L.lbm_set_velocity(self.ctx, inst, ux, uy, uz)

    def set_diffusion(self, D: torch.Tensor, inst: int = 0) -> None:
        L.lbm_set_diffusion(self.ctx, inst, D)

    def set_dirichlet(self, phi_b: torch.Tensor, inst: int = 0) -> None:
        self._keep_bc = phi_b
        L.lbm_set_dirichlet(self.ctx, inst, phi_b)

    def macros(self, inst: int = 0, ref: Optional[torch.Tensor] = None, want_phi: bool = False,
               raise_nonfinite: bool = True):
        phi = torch.empty(self._shape(inst), dtype=torch.float64, device="cuda") if want_phi else None
        stats = L.lbm_macros(self.ctx, inst, phi, ref, raise_nonfinite)
        return (stats, phi) if want_phi else stats

    def populations(self, inst: int = 0) -> torch.Tensor:
        out = torch.empty((self._q(inst),) + self._shape(inst), dtype=torch.float64, device="cuda")
        L.lbm_populations(self.ctx, inst, out)
        return out

    def state_save(self, inst: int = 0) -> torch.Tensor:
        buf = torch.empty(L.lbm_state_bytes(self.ctx, inst), dtype=torch.uint8, device="cuda")
        L.lbm_state_save(self.ctx, inst, buf)
        return buf

    def state_load(self, buf: torch.Tensor, step: int, inst: int = 0) -> None:
        L.lbm_state_load(self.ctx, inst, buf, step)

    def set_launch(self, rows: int, xcd_remap: int = 1, inst: int = -1, tile_width: int = 64,
                   max_waves: int = 0, xcd_rows: int = 0, stores: int = 0, fuse: int = 1) -> None:
        L.lbm_set_launch(self.ctx, inst, rows, xcd_remap, tile_width, max_waves, xcd_rows, stores, fuse)

    def get_launch(self, inst: int = 0) -> dict:
        return L.lbm_get_launch(self.ctx, inst)

    def set_batch(self, policy: int, blocks: int = 0, max_waves: int = 0) -> None:
        L.lbm_set_batch(self.ctx, policy, blocks, max_waves)

    def get_batch(self) -> dict:
        return L.lbm_get_batch(self.ctx)

    def close(self) -> None:
        if self.ctx is not None:
            L.lbm_free(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
