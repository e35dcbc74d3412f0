"""Seeded synthetic inputs for the TRT-R D2Q9 solver and its oracle.

This module is shared by the product, the oracle-based tests and the benchmark.  It holds problem
definitions only -- lattice coordinates, velocity, diffusion and source fields, initial pulses, the
closed-form solutions they are measured against, and seeded parameter draws -- and none of the lattice
Boltzmann arithmetic.

Workloads (all on periodic, vertex-centred lattices x_j = lo + j*dx, j = 0..N-1):

* ``rotating_pulse``: Gaussian pulse in the solid-body rotation u = (-U0 y, U0 x) on [-1, 1]^2 with
  constant or variable D and no source.  With solid-body rotation the advection commutes with the
  Laplacian, so on an unbounded plane phi(x, t) = s0^2/s^2 exp(-|x - R(U0 t) x_c0|^2 / (2 s^2)),
  s^2 = s0^2 + 2 D t (constant D).
* ``x1_problem``: the benchmark of Sec. 3 (rotating flow u = (-y, x) on [-2 pi, 2 pi]^2, phi0 =
  exp(-(x^2 + 3 y^2)), the source S of Sec. 3 and the closed form phi = exp(-(x^2 + 3 y^2 + 2 kappa t)))
  on a periodic lattice with the diffusive scaling dx^2/dt = 0.16 pi^2 of Sec. 3.2.
* ``batched_instances``: seeded draws of many pulse instances of uneven sizes and coefficients.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

PI = math.pi


def lattice_coords(n: int, lo: float, hi: float):
    """Vertex-centred periodic coordinates: x_j = lo + j*dx, dx = (hi - lo)/n."""
    dx = (hi - lo) / n
    return lo + dx * np.arange(n, dtype=np.float64), dx


def mesh(nx: int, ny: int, lo: float, hi: float):
    x, dx = lattice_coords(nx, lo, hi)
    y, dy = lattice_coords(ny, lo, hi)
    Y, X = np.meshgrid(y, x, indexing="ij")  # [ny, nx]
    return X, Y, dx


def variable_D(X, Y, D0: float = 1e-3, amp: float = 0.5):
    """D(x) = D0 (1 + amp sin(pi x) sin(pi y)) -- periodic on [-1, 1]^2."""
    return D0 * (1.0 + amp * np.sin(PI * X) * np.sin(PI * Y))


def pulse_exact(X, Y, t: float, U0: float, D: float, xc0: float, yc0: float, sigma0: float):
    """Closed-form rotating Gaussian pulse on the unbounded plane (constant D, no source)."""
    a = U0 * t
    xc = math.cos(a) * xc0 - math.sin(a) * yc0
    yc = math.sin(a) * xc0 + math.cos(a) * yc0
    s2 = sigma0 * sigma0 + 2.0 * D * t
    r2 = (X - xc) ** 2 + (Y - yc) ** 2
    return (sigma0 * sigma0 / s2) * np.exp(-r2 / (2.0 * s2))


@dataclass
class PulseConfig:
    """Rotating-pulse workload on [-1, 1]^2, c = dx/dt fixed (acoustic scaling by default)."""
    N: int = 64
    steps: int = 160
    U0: float = PI
    D: float = 1e-3
    D_variable: bool = False    # D(x) = D (1 + 0.5 sin(pi x) sin(pi y))
    sigma0: float = 0.1
    xc0: float = 0.5
    yc0: float = 0.0
    c: float = 10.0              # lattice speed dx/dt
    lam: float = 0.25            # magic parameter
    dt_override: Optional[float] = None   # diffusive scaling: give dt explicitly

    @property
    def dx(self) -> float:
        return 2.0 / self.N

    @property
    def dt(self) -> float:
        return self.dt_override if self.dt_override is not None else self.dx / self.c

    @property
    def t_end(self) -> float:
        return self.steps * self.dt


def rotating_pulse(cfg: PulseConfig) -> dict:
    """Fields (FP64, [N, N]) and scalars of one rotating-pulse instance."""
    X, Y, dx = mesh(cfg.N, cfg.N, -1.0, 1.0)
    ux = -cfg.U0 * Y
    uy = cfg.U0 * X
    phi0 = pulse_exact(X, Y, 0.0, cfg.U0, cfg.D, cfg.xc0, cfg.yc0, cfg.sigma0)
    D = variable_D(X, Y, cfg.D) if cfg.D_variable else None
    return dict(X=X, Y=Y, dx=dx, dt=cfg.dt, lam=cfg.lam, D_const=cfg.D, D=D, ux=ux, uy=uy, phi0=phi0,
                nx=cfg.N, ny=cfg.N)


def pulse_reference(cfg: PulseConfig, fields: dict, steps: Optional[int] = None):
    t = (cfg.steps if steps is None else steps) * cfg.dt
    return pulse_exact(fields["X"], fields["Y"], t, cfg.U0, cfg.D, cfg.xc0, cfg.yc0, cfg.sigma0)


# Named configurations (one periodic pulse instance each).
C1 = PulseConfig(N=64, steps=160)                                   # 64^2, FP64 parity, t = 0.5
C2 = PulseConfig(N=2048, steps=3200)                                # 2048^2, t = 0.3125
C3 = PulseConfig(N=8192, steps=1000, D_variable=True)               # 8192^2, variable D
C5 = PulseConfig(N=512, steps=400)                                  # adjoint forward


def refinement(N: int, scaling: str = "acoustic", t_end: float = 0.3125, N0: int = 256,
               base: PulseConfig = C2) -> PulseConfig:
    """Grid-refinement member: acoustic (c fixed) or diffusive (dx^2/dt fixed at its N0 value)."""
    dx = 2.0 / N
    if scaling == "acoustic":
        dt = dx / base.c
    elif scaling == "diffusive":
        dx0 = 2.0 / N0
        dt = (dx0 / base.c) * (dx / dx0) ** 2
    else:
        raise ValueError(scaling)
    steps = int(round(t_end / dt))
    return replace(base, N=N, steps=steps, dt_override=dt)


# ---- the benchmark of Sec. 3 on a periodic lattice ------------------------------------------

def x1_problem(N: int, kappa: float, lam: float = 1.0 / 12.0, t_end: float = 1.0, dirichlet: bool = False):
    """Rotating-flow pulse held stationary by a source (Sec. 3) on [-2pi, 2pi]^2 with dx = 4 pi / N.

    Periodic proxy (N nodes per axis) or, with ``dirichlet``, the N + 1 nodes x_j = -2 pi + j dx,
    j = 0..N, whose first and last rows and columns carry the closed form as Dirichlet values.
    Diffusive scaling dx^2/dt = 0.16 pi^2 (Sec. 3.2).  Returns a dict with fields, a function
    ``source(t) -> (S, dSdt)`` and ``exact(t)``."""
    L = 4.0 * PI
    if dirichlet:
        x = -2.0 * PI + (4.0 * PI / N) * np.arange(N + 1)
        Y, X = np.meshgrid(x, x, indexing="ij")
        dx = 4.0 * PI / N
    else:
        X, Y, dx = mesh(N, N, -2.0 * PI, 2.0 * PI)
    dt = dx * dx / (0.16 * PI * PI)
    steps = int(round(t_end / dt))
    ux = -Y
    uy = X.copy()
    q = X * X + 3.0 * Y * Y
    base = (6.0 * kappa - 4.0 * X * Y - 4.0 * kappa * (X * X + 9.0 * Y * Y)) * np.exp(-q)

    def source(t: float):
        S = base * math.exp(-2.0 * kappa * t)
        return S, -2.0 * kappa * S

    def exact(t: float):
        return np.exp(-(q + 2.0 * kappa * t))

    n = X.shape[0]
    return dict(X=X, Y=Y, dx=dx, dt=dt, steps=steps, lam=lam, D_const=kappa, ux=ux, uy=uy,
                phi0=np.exp(-q), source=source, exact=exact, nx=n, ny=n, L=L)


# ---- D3Q19: the rotating pulse in three dimensions ---------------------------------------------

def mesh3(nx: int, ny: int, nz: int, lo: float, hi: float):
    """Vertex-centred periodic coordinates, arrays [nz, ny, nx]."""
    x, dx = lattice_coords(nx, lo, hi)
    y, _ = lattice_coords(ny, lo, hi)
    z, _ = lattice_coords(nz, lo, hi)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z, dx


def pulse3_exact(X, Y, Z, t: float, U0: float, D: float, xc0: float, yc0: float, zc0: float, sigma0: float):
    """Closed-form Gaussian pulse in the solid-body rotation about the z axis (constant D, no source,
    unbounded space): phi = (s0^2/s^2)^(3/2) exp(-|x - R(U0 t) x_c0|^2 / (2 s^2)), s^2 = s0^2 + 2 D t."""
    a = U0 * t
    xc = math.cos(a) * xc0 - math.sin(a) * yc0
    yc = math.sin(a) * xc0 + math.cos(a) * yc0
    s2 = sigma0 * sigma0 + 2.0 * D * t
    r2 = (X - xc) ** 2 + (Y - yc) ** 2 + (Z - zc0) ** 2
    return (sigma0 * sigma0 / s2) ** 1.5 * np.exp(-r2 / (2.0 * s2))


def rotating_pulse3(cfg: PulseConfig) -> dict:
    """D3Q19 rotating pulse on [-1, 1]^3 (N^3 nodes): u = (-U0 y, U0 x, 0), centre (xc0, yc0, 0)."""
    X, Y, Z, dx = mesh3(cfg.N, cfg.N, cfg.N, -1.0, 1.0)
    u = np.stack([-cfg.U0 * Y, cfg.U0 * X, np.zeros_like(X)])
    phi0 = pulse3_exact(X, Y, Z, 0.0, cfg.U0, cfg.D, cfg.xc0, cfg.yc0, 0.0, cfg.sigma0)
    return dict(X=X, Y=Y, Z=Z, dx=dx, dt=cfg.dt, lam=cfg.lam, D_const=cfg.D, u=u, phi0=phi0, n=cfg.N)


def pulse3_reference(cfg: PulseConfig, fields: dict, steps: Optional[int] = None):
    t = (cfg.steps if steps is None else steps) * cfg.dt
    return pulse3_exact(fields["X"], fields["Y"], fields["Z"], t, cfg.U0, cfg.D, cfg.xc0, cfg.yc0, 0.0, cfg.sigma0)


C6 = PulseConfig(N=256, steps=400)  # D3Q19 rotating pulse, 256^3, t = 0.3125


# ---- batched instances -----------------------------------------------------------------------

@dataclass
class Instance:
    N: int
    D: float
    U0: float
    sigma0: float
    theta: float
    steps: int = 2000
    c: float = 10.0
    lam: float = 0.25

    @property
    def config(self) -> PulseConfig:
        return PulseConfig(N=self.N, steps=self.steps, U0=self.U0, D=self.D, sigma0=self.sigma0,
                           xc0=0.5 * math.cos(self.theta), yc0=0.5 * math.sin(self.theta), c=self.c,
                           lam=self.lam)


def batched_instances(n: int = 256, seed: int = 231210316, steps: int = 2000, n_lo: int = 32,
                      n_hi: int = 512) -> list:
    """Seeded draws: N log-uniform in [n_lo, n_hi] (rounded), D log-uniform in [1e-4, 1e-2],
    U0 uniform in [pi/2, 2 pi], sigma0 uniform in [0.05, 0.15], centre at radius 0.5 at a uniform
    angle.  Vectors are drawn in that order."""
    rng = np.random.default_rng(seed)
    Ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n))).astype(int)
    Ds = np.exp(rng.uniform(math.log(1e-4), math.log(1e-2), n))
    U0s = rng.uniform(0.5 * PI, 2.0 * PI, n)
    sig = rng.uniform(0.05, 0.15, n)
    th = rng.uniform(0.0, 2.0 * PI, n)
    return [Instance(int(Ns[k]), float(Ds[k]), float(U0s[k]), float(sig[k]), float(th[k]), steps)
            for k in range(n)]


def random_populations(shape, seed: int, lo: float = 0.0, hi: float = 1.0):
    """Seeded uniform random values (used as arbitrary population states in tests)."""
    return np.random.default_rng(seed).uniform(lo, hi, shape)


# ---- D(x) on a control grid (gradient workloads) ---------------------------------------------

def bspline_matrix(n_nodes: int, n_ctrl: int) -> np.ndarray:
    """Periodic uniform cubic B-spline basis: B[j, a] = b3((j/n_nodes - a/n_ctrl) * n_ctrl) with the
    argument wrapped to the period; b3 is the cubic B-spline (a positive partition of unity)."""
    t = np.arange(n_nodes)[:, None] / n_nodes * n_ctrl - np.arange(n_ctrl)[None, :]
    t = (t + n_ctrl / 2.0) % n_ctrl - n_ctrl / 2.0
    a = np.abs(t)
    return np.where(a < 1.0, (4.0 - 6.0 * a * a + 3.0 * a ** 3) / 6.0,
                    np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def D_from_control(theta: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """D[y, x] = sum_ab By[y, a] theta[a, b] Bx[x, b] (bicubic periodic B-spline surface)."""
    By = bspline_matrix(ny, theta.shape[0])
    Bx = bspline_matrix(nx, theta.shape[1])
    return By @ theta @ Bx.T


def control_theta(n_ctrl: int = 32, seed: int = 231210316 + 5, D0: float = 1e-3, amp: float = 0.3) -> np.ndarray:
    """Seeded control values D0 (1 + amp (2U - 1)) on an n_ctrl x n_ctrl grid."""
    rng = np.random.default_rng(seed)
    return D0 * (1.0 + amp * (2.0 * rng.uniform(0.0, 1.0, (n_ctrl, n_ctrl)) - 1.0))


C5_N, C5_STEPS, C5_CTRL = 512, 400, 32  # 512^2 pulse, 400 steps, 32 x 32 control grid
