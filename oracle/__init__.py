"""Plain FP64 CPU oracle of the TRT-R lattice Boltzmann step (arXiv:2312.10316).

TEST INFRASTRUCTURE ONLY.  This package is the checker, not the product: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no
code with the HIP library (``paper_2312_10316_amd``) and never imports it.

The arithmetic lives in ``lbm_oracle.c`` (plain C, compiled with ``gcc -O2 -ffp-contract=off``, no
fast-math, twice: FP64 and FP64-complex for complex-step derivatives) and, for the D3Q19 and D3Q27
lattices, in ``lbm_oracle_3d.c`` (FP64).  This module only marshals
numpy arrays.  Reductions (mass, the RMS error of Sec. 3, Eq. (33)) are computed here with
``math.fsum`` (correctly rounded sums), in the definitions' own terms.

Array layout: populations ``g[9, ny, nx]`` (pre-collision, time t_n); fields ``[ny, nx]``; node
(j, k) is ``[k, j]``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRC3 = os.path.join(_HERE, "lbm_oracle_3d.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_LIB_OMP = os.path.join(_HERE, "liblbm_oracle_omp.so")

AUX_LOCAL, AUX_FLUX, AUX_NONE = 0, 1, 2
BC_PERIODIC, BC_NEE, BC_WALLS = 0, 1, 2


_CFLAGS = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-Wall"]


def _stale(lib: str) -> bool:
    return not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(_SRC), os.path.getmtime(_SRC3))


def build(force: bool = False) -> str:
    """Compile the oracle into its shared objects; returns the path of the main one.

    ``liblbm_oracle.so`` holds the FP64 build, the complex-step build and the 3D oracle, all
    single-threaded.  ``liblbm_oracle_omp.so`` is the FP64 D2Q9 source compiled once more with
    ``-fopenmp`` (rows of a step split over host threads; bitwise the same results), used only to time
    the oracle on every host core and to write stored expected values of large cases."""
    if force or _stale(_LIB):
        objs = []
        for tag, src, extra in (("r", _SRC, []), ("z", _SRC, ["-DORC_COMPLEX"]), ("3", _SRC3, [])):
            obj = os.path.join(_HERE, f"_lbm_oracle_{tag}.o")
            subprocess.run(_CFLAGS + ["-c", src, "-o", obj] + extra, check=True)
            objs.append(obj)
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-shared", "-o", tmp] + objs + ["-lm"], check=True)
        os.replace(tmp, _LIB)
        for o in objs:
            os.remove(o)
    if force or _stale(_LIB_OMP):
        tmp = _LIB_OMP + ".tmp"
        subprocess.run(_CFLAGS + ["-fopenmp", "-shared", _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_OMP)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("lambda_", ctypes.c_double), ("D_const", ctypes.c_double),
                ("aux", ctypes.c_int), ("boundary", ctypes.c_int), ("tau3", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        dbl, i32 = ctypes.c_double, ctypes.c_int
        zc = ctypes.c_double * 2  # C99 double _Complex is passed like struct {double re, im}
        lib.orc_lattice.argtypes = [P, P, P]
        lib.orc_equilibrium.argtypes = [dbl, dbl, dbl, dbl, P]
        lib.orc_collide.argtypes = [P, dbl, dbl, dbl, dbl, dbl, P]
        lib.orc_collide_mrt.argtypes = [P, dbl, dbl, dbl, dbl, dbl, dbl, P]
        lib.orc_relaxation.argtypes = [dbl, dbl, dbl, dbl, P, P]
        for pre in ("orc_", "orc_z_"):
            getattr(lib, pre + "init").argtypes = [P, P, P, P, P]
            getattr(lib, pre + "phi").argtypes = [P, P, P]
            getattr(lib, pre + "step").argtypes = [P, P, P, P, P, P, P, P, P]
            getattr(lib, pre + "run").argtypes = [P, P, i32, P, P, P, P, P, P, P]
            getattr(lib, pre + "apply_nee").argtypes = [P, P, P, P, P]
        lib.orc3_lattice.argtypes = [i32, P, P, P, P]
        lib.orc3_equilibrium.argtypes = [i32, dbl, P, dbl, P]
        lib.orc3_collide.argtypes = [i32, P, P, dbl, dbl, dbl, P]
        lib.orc3_init.argtypes = [P, P, P, P]
        lib.orc3_phi.argtypes = [P, P, P]
        lib.orc3_step.argtypes = [P, P, P, P, P, P, P]
        lib.orc3_run.argtypes = [P, P, i32, P, P, P, P, P]
        del zc
        _lib = lib
    return _lib


@dataclass
class Problem:
    """One instance: lattice, time step, magic parameter, constant D, aux-term form, edge treatment."""
    nx: int
    ny: int
    dx: float
    dt: float
    lam: float
    D_const: float = 0.0
    aux: int = AUX_LOCAL
    boundary: int = BC_PERIODIC   # BC_NEE: one-sided derivatives of u across the edges (apply_nee per step);
                                  # BC_WALLS: halfway anti-bounce-back walls below row 0 and above row ny-1
    tau3: float = 0.0             # MRT-R third-order relaxation time; 0 (or 1): TRT-R

    def _c(self) -> _Problem:
        return _Problem(self.nx, self.ny, self.dx, self.dt, self.lam, self.D_const, self.aux, self.boundary,
                        self.tau3)

    @property
    def c(self) -> float:
        return self.dx / self.dt


def _arr(a, shape, cplx):
    dt = np.complex128 if cplx else np.float64
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=dt), shape))
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def lattice():
    """(ex[9], ey[9], w[9]) in the oracle's velocity order (lattice units, e = c * (ex, ey))."""
    lib = _load()
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    w = np.zeros(9, np.float64)
    lib.orc_lattice(_ptr(ex), _ptr(ey), _ptr(w))
    return ex.astype(np.int64), ey.astype(np.int64), w


def equilibrium(phi: float, ux: float, uy: float, c: float) -> np.ndarray:
    out = np.zeros(9)
    _load().orc_equilibrium(phi, ux, uy, c, _ptr(out))
    return out


def collide(g, ux: float, uy: float, tau1: float, tau2: float, c: float) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros(9)
    _load().orc_collide(_ptr(g), ux, uy, tau1, tau2, c, _ptr(out))
    return out


def collide_mrt(g, ux: float, uy: float, tau1: float, tau2: float, tau3: float, c: float) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros(9)
    _load().orc_collide_mrt(_ptr(g), ux, uy, tau1, tau2, tau3, c, _ptr(out))
    return out


_lib_omp = None


def _load_omp():
    global _lib_omp
    if _lib_omp is None:
        build()
        lib = ctypes.CDLL(_LIB_OMP)
        P = ctypes.c_void_p
        lib.orc_run.argtypes = [P, P, ctypes.c_int, P, P, P, P, P, P, P]
        lib.orc_threads.argtypes = [ctypes.c_int]
        lib.orc_threads.restype = ctypes.c_int
        _lib_omp = lib
    return _lib_omp


def run_threads(p: Problem, g, nsteps: int, ux, uy, D=None, S=None, dSdt=None, threads: int = 0):
    """``run`` (FP64, no walls) on ``threads`` host threads (0: every core OpenMP sees), through the
    OpenMP build of the same source; returns (final populations, threads used).  Bitwise equal to
    ``run``."""
    lib = _load_omp()
    used = lib.orc_threads(int(threads))
    g = np.array(g, dtype=np.float64, copy=True, order="C")
    ux, uy, D, S, dSdt = _fields(p, ux, uy, D, S, dSdt, False)
    if p.boundary == BC_WALLS:
        raise ValueError("run_threads covers lattices without walls")
    work = np.empty_like(g)
    pc = p._c()
    lib.orc_run(ctypes.byref(pc), _ptr(g), int(nsteps), _ptr(ux), _ptr(uy), _ptr(D), _ptr(S), _ptr(dSdt),
                None, _ptr(work))
    return g, used


def relaxation(kappa: float, dx: float, dt: float, lam: float):
    t1 = ctypes.c_double()
    t2 = ctypes.c_double()
    _load().orc_relaxation(kappa, dx, dt, lam, ctypes.byref(t1), ctypes.byref(t2))
    return t1.value, t2.value


def _fields(p: Problem, ux, uy, D, S, dSdt, cplx):
    sh = (p.ny, p.nx)
    ux = _arr(ux, sh, cplx)
    uy = _arr(uy, sh, cplx)
    D = None if D is None else _arr(D, sh, cplx)
    S = None if S is None else _arr(S, sh, cplx)
    dSdt = None if dSdt is None else _arr(dSdt, sh, cplx)
    return ux, uy, D, S, dSdt


def init(p: Problem, phi0, ux, uy, cplx: bool = False) -> np.ndarray:
    """g_i = g_eq_i(phi0, u) (the initial condition of Sec. 3)."""
    lib = _load()
    sh = (p.ny, p.nx)
    phi0 = _arr(phi0, sh, cplx)
    ux, uy, *_ = _fields(p, ux, uy, None, None, None, cplx)
    g = np.zeros((9,) + sh, np.complex128 if cplx else np.float64)
    pc = p._c()
    (lib.orc_z_init if cplx else lib.orc_init)(ctypes.byref(pc), _ptr(phi0), _ptr(ux), _ptr(uy), _ptr(g))
    return g


def phi(p: Problem, g) -> np.ndarray:
    lib = _load()
    cplx = np.iscomplexobj(g)
    g = np.ascontiguousarray(g, dtype=np.complex128 if cplx else np.float64)
    out = np.zeros((p.ny, p.nx), g.dtype)
    pc = p._c()
    (lib.orc_z_phi if cplx else lib.orc_phi)(ctypes.byref(pc), _ptr(g), _ptr(out))
    return out


def _walls(p: Problem, phi_b, cplx):
    if p.boundary != BC_WALLS:
        return None
    if phi_b is None:
        raise ValueError("walls need phi_b (rows 0 and ny-1 hold the bottom and top wall values)")
    return _arr(phi_b, (p.ny, p.nx), cplx)


def step(p: Problem, g, ux, uy, D=None, S=None, dSdt=None, phi_b=None) -> np.ndarray:
    """One step of Eq. (14) on a copy of g; returns the new pre-collision populations.  For walls,
    phi_b [ny, nx] holds the wall values (rows 0 and ny-1) at the new time level."""
    lib = _load()
    cplx = np.iscomplexobj(g) or any(np.iscomplexobj(a) for a in (ux, uy, D, S, dSdt, phi_b) if a is not None)
    g = np.ascontiguousarray(g, dtype=np.complex128 if cplx else np.float64)
    ux, uy, D, S, dSdt = _fields(p, ux, uy, D, S, dSdt, cplx)
    pb = _walls(p, phi_b, cplx)
    out = np.empty_like(g)
    pc = p._c()
    (lib.orc_z_step if cplx else lib.orc_step)(ctypes.byref(pc), _ptr(g), _ptr(out), _ptr(ux), _ptr(uy),
                                               _ptr(D), _ptr(S), _ptr(dSdt), _ptr(pb))
    return out


def run(p: Problem, g, nsteps: int, ux, uy, D=None, S=None, dSdt=None, phi_b=None) -> np.ndarray:
    """nsteps steps with fixed u, D, S, dS/dt (and wall values); returns the final populations
    (input untouched)."""
    lib = _load()
    cplx = np.iscomplexobj(g) or any(np.iscomplexobj(a) for a in (ux, uy, D, S, dSdt, phi_b) if a is not None)
    g = np.array(g, dtype=np.complex128 if cplx else np.float64, copy=True, order="C")
    ux, uy, D, S, dSdt = _fields(p, ux, uy, D, S, dSdt, cplx)
    pb = _walls(p, phi_b, cplx)
    work = np.empty_like(g)
    pc = p._c()
    (lib.orc_z_run if cplx else lib.orc_run)(ctypes.byref(pc), _ptr(g), int(nsteps), _ptr(ux), _ptr(uy),
                                             _ptr(D), _ptr(S), _ptr(dSdt), _ptr(pb), _ptr(work))
    return g


def apply_nee(p: Problem, g, ux, uy, phi_b) -> np.ndarray:
    """Dirichlet edges by non-equilibrium extrapolation (the boundary scheme of Sec. 3), applied to
    a copy of the pre-collision state g; phi_b [ny, nx] holds the boundary values."""
    lib = _load()
    cplx = np.iscomplexobj(g) or np.iscomplexobj(phi_b)
    g = np.array(g, dtype=np.complex128 if cplx else np.float64, copy=True, order="C")
    ux, uy, *_ = _fields(p, ux, uy, None, None, None, cplx)
    pb = _arr(phi_b, (p.ny, p.nx), cplx)
    pc = p._c()
    (lib.orc_z_apply_nee if cplx else lib.orc_apply_nee)(ctypes.byref(pc), _ptr(g), _ptr(ux), _ptr(uy), _ptr(pb))
    return g


# ---- diagnostics: the definitions written out with correctly rounded sums ---------------------

def mass(phi_field) -> float:
    """sum_x phi (correctly rounded)."""
    return math.fsum(np.asarray(phi_field, dtype=np.float64).ravel().tolist())


def rms_error(phi_num, phi_ref) -> float:
    """E_r = sqrt(sum |phi_num - phi_ref|^2 / (Nx Ny)), Sec. 3, Eq. (33)."""
    d = (np.asarray(phi_num, np.float64) - np.asarray(phi_ref, np.float64)).ravel()
    return math.sqrt(math.fsum((d * d).tolist()) / d.size)


def l2_rel_error(phi_num, phi_ref) -> float:
    d = (np.asarray(phi_num, np.float64) - np.asarray(phi_ref, np.float64)).ravel()
    r = np.asarray(phi_ref, np.float64).ravel()
    return math.sqrt(math.fsum((d * d).tolist()) / math.fsum((r * r).tolist()))


def max_abs_error(phi_num, phi_ref) -> float:
    return float(np.max(np.abs(np.asarray(phi_num, np.float64) - np.asarray(phi_ref, np.float64))))


# ---- D3Q19 / D3Q27 -------------------------------------------------------------------------------

class _Problem3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("lambda_", ctypes.c_double), ("D_const", ctypes.c_double),
                ("aux", ctypes.c_int), ("q", ctypes.c_int)]


@dataclass
class Problem3:
    """One periodic D3Q19 (q = 19) or D3Q27 (q = 27) instance.  Arrays: populations g[q, nz, ny, nx];
    u[3, nz, ny, nx]; scalar fields [nz, ny, nx]; node (j, k, l) is [l, k, j]."""
    nx: int
    ny: int
    nz: int
    dx: float
    dt: float
    lam: float
    D_const: float = 0.0
    aux: int = AUX_LOCAL
    q: int = 19

    def __post_init__(self):
        if self.q not in (19, 27):
            raise ValueError("q must be 19 or 27")

    def _c(self) -> _Problem3:
        return _Problem3(self.nx, self.ny, self.nz, self.dx, self.dt, self.lam, self.D_const, self.aux, self.q)

    @property
    def c(self) -> float:
        return self.dx / self.dt

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


def _q(q: int) -> int:
    if q not in (19, 27):
        raise ValueError("q must be 19 or 27")
    return q


def lattice3(q: int = 19):
    """(ex[q], ey[q], ez[q], w[q]) of the D3Q19 or D3Q27 oracle (lattice units)."""
    lib = _load()
    e = [np.zeros(_q(q), np.int32) for _ in range(3)]
    w = np.zeros(q, np.float64)
    lib.orc3_lattice(q, *(_ptr(a) for a in e), _ptr(w))
    return tuple(a.astype(np.int64) for a in e) + (w,)


def equilibrium3(phi: float, u, c: float, q: int = 19) -> np.ndarray:
    out = np.zeros(_q(q))
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _load().orc3_equilibrium(q, phi, _ptr(uu), c, _ptr(out))
    return out


def collide3(g, u, tau1: float, tau2: float, c: float) -> np.ndarray:
    """TRT-R collision of one node; the lattice follows from len(g) (19 or 27)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    q = _q(len(g))
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(q)
    _load().orc3_collide(q, _ptr(g), _ptr(uu), tau1, tau2, c, _ptr(out))
    return out


def _f3(p: Problem3, a):
    return None if a is None else np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), p.shape))


def _u3(p: Problem3, u):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(u, np.float64), (3,) + p.shape))


def _g3(p: Problem3, g):
    g = np.ascontiguousarray(g, dtype=np.float64)
    if g.shape != (p.q,) + p.shape:
        raise ValueError(f"populations must have shape {(p.q,) + p.shape}, got {g.shape}")
    return g


def init3(p: Problem3, phi0, u) -> np.ndarray:
    g = np.zeros((p.q,) + p.shape)
    pc = p._c()
    _load().orc3_init(ctypes.byref(pc), _ptr(_f3(p, phi0)), _ptr(_u3(p, u)), _ptr(g))
    return g


def phi3(p: Problem3, g) -> np.ndarray:
    g = _g3(p, g)
    out = np.zeros(p.shape)
    pc = p._c()
    _load().orc3_phi(ctypes.byref(pc), _ptr(g), _ptr(out))
    return out


def step3(p: Problem3, g, u, D=None, S=None, dSdt=None) -> np.ndarray:
    g = _g3(p, g)
    out = np.empty_like(g)
    pc = p._c()
    _load().orc3_step(ctypes.byref(pc), _ptr(g), _ptr(out), _ptr(_u3(p, u)), _ptr(_f3(p, D)), _ptr(_f3(p, S)),
                      _ptr(_f3(p, dSdt)))
    return out


def run3(p: Problem3, g, nsteps: int, u, D=None, S=None, dSdt=None) -> np.ndarray:
    g = np.array(_g3(p, g), dtype=np.float64, copy=True, order="C")
    work = np.empty_like(g)
    pc = p._c()
    _load().orc3_run(ctypes.byref(pc), _ptr(g), int(nsteps), _ptr(_u3(p, u)), _ptr(_f3(p, D)), _ptr(_f3(p, S)),
                     _ptr(_f3(p, dSdt)), _ptr(work))
    return g
