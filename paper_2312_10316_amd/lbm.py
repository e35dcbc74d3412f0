"""Python binding of the C ABI in ``include/lbm.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls and converts torch tensors to device
pointers; all computation runs in the HIP kernels of ``liblbm.so``.  There is no fallback: if the
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_E_ARG, LBM_E_HIP, LBM_E_STATE, LBM_E_NONFINITE, LBM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
LBM_STORE_F64, LBM_STORE_F32, LBM_STORE_F16S, LBM_STORE_F16SR = 0, 1, 2, 3
LBM_MATH_F64, LBM_MATH_F32 = 0, 1
LBM_AUX_LOCAL, LBM_AUX_FLUX, LBM_AUX_NONE = 0, 1, 2
LBM_BC_PERIODIC, LBM_BC_NEE, LBM_BC_WALLS = 0, 1, 2
LBM_LATTICE_D2Q9, LBM_LATTICE_D3Q19, LBM_LATTICE_D3Q27 = 0, 1, 2
LATTICE_Q = {LBM_LATTICE_D2Q9: 9, LBM_LATTICE_D3Q19: 19, LBM_LATTICE_D3Q27: 27}

# names of the population storage / arithmetic combinations
MODES = {
    "f64": (LBM_STORE_F64, LBM_MATH_F64),
    "f64s_f32m": (LBM_STORE_F64, LBM_MATH_F32),
    "f32": (LBM_STORE_F32, LBM_MATH_F32),
    "f16s": (LBM_STORE_F16S, LBM_MATH_F32),
    "f16sr": (LBM_STORE_F16SR, LBM_MATH_F32),  # the F16S code with stochastic rounding
}
STORE_BYTES = {LBM_STORE_F64: 8, LBM_STORE_F32: 4, LBM_STORE_F16S: 2, LBM_STORE_F16SR: 2}


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"liblbm status {status}: {message}")
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("D_const", ctypes.c_double), ("store", ctypes.c_int32),
                ("math", ctypes.c_int32), ("aux", ctypes.c_int32), ("scale_log2", ctypes.c_int32),
                ("phi_ref", ctypes.c_double), ("boundary", ctypes.c_int32), ("round_seed", ctypes.c_int32),
                ("tau3", ctypes.c_double), ("lattice", ctypes.c_int32), ("nz", ctypes.c_int32)]


class lbm_fields(ctypes.Structure):
    _fields_ = [("phi0", ctypes.c_void_p), ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("D", ctypes.c_void_p),
                ("uz", ctypes.c_void_p)]


class lbm_stats(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("rms_err", ctypes.c_double), ("l2_rel_err", ctypes.c_double),
                ("max_abs_err", ctypes.c_double), ("max_abs_phi", ctypes.c_double), ("nonfinite", ctypes.c_int64),
                ("step", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_launch(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("xcd_remap", ctypes.c_int32), ("tile_width", ctypes.c_int32),
                ("max_waves", ctypes.c_int32), ("xcd_rows", ctypes.c_int32), ("stores", ctypes.c_int32),
                ("fuse", ctypes.c_int32)]


class lbm_batch(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("blocks", ctypes.c_int32), ("max_waves", ctypes.c_int32)]


LBM_BATCH_SERIAL, LBM_BATCH_FLAT, LBM_BATCH_STRIDED, LBM_BATCH_LPT = 0, 1, 2, 3

EXPORTS = ["lbm_workspace_size", "lbm_init", "lbm_step", "lbm_set_velocity", "lbm_set_dirichlet", "lbm_macros", "lbm_populations", "lbm_state_bytes",
           "lbm_state_save", "lbm_state_load", "lbm_set_launch", "lbm_get_launch", "lbm_set_batch", "lbm_get_batch",
           "lbm_adjoint_bytes", "lbm_adjoint_seed", "lbm_adjoint_step", "lbm_adjoint_init", "lbm_bench_copy", "lbm_free",
           "lbm_pitch", "lbm_last_error", "lbm_abi_version", "lbm_set_diffusion", "lbm_adjoint_segment",
           "lbm_bench_copy_cached", "lbm_macros_static"]


def pitch_of(p: "lbm_params") -> int:
    """Row pitch (elements) of the library's layouts for instance parameters p (lbm_pitch)."""
    out = ctypes.c_int64()
    _check(lib().lbm_pitch(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built (run __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(path)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.lbm_workspace_size.argtypes = [I32, ctypes.POINTER(lbm_params), ctypes.POINTER(SZ)]
    lib.lbm_init.argtypes = [ctypes.POINTER(P), I32, ctypes.POINTER(lbm_params), ctypes.POINTER(lbm_fields), P, SZ, P]
    lib.lbm_step.argtypes = [P, I32, PP, PP, PP, PP]
    lib.lbm_macros.argtypes = [P, I32, P, P, ctypes.POINTER(lbm_stats)]
    lib.lbm_macros_static.argtypes = [P, I32, P, P, ctypes.POINTER(lbm_stats)]
    lib.lbm_set_dirichlet.argtypes = [P, I32, P]
    lib.lbm_set_velocity.argtypes = [P, I32, P, P, P]
    lib.lbm_populations.argtypes = [P, I32, P]
    lib.lbm_state_bytes.argtypes = [P, I32, ctypes.POINTER(SZ)]
    lib.lbm_pitch.argtypes = [ctypes.POINTER(lbm_params), ctypes.POINTER(I64)]
    lib.lbm_state_save.argtypes = [P, I32, P]
    lib.lbm_state_load.argtypes = [P, I32, P, I64]
    lib.lbm_set_launch.argtypes = [P, I32, ctypes.POINTER(lbm_launch)]
    lib.lbm_get_launch.argtypes = [P, I32, ctypes.POINTER(lbm_launch)]
    lib.lbm_set_batch.argtypes = [P, ctypes.POINTER(lbm_batch)]
    lib.lbm_get_batch.argtypes = [P, ctypes.POINTER(lbm_batch)]
    lib.lbm_adjoint_bytes.argtypes = [P, I32, ctypes.POINTER(SZ)]
    lib.lbm_adjoint_seed.argtypes = [P, I32, P, P]
    lib.lbm_adjoint_step.argtypes = [P, I32, P, P, P, P]
    lib.lbm_adjoint_init.argtypes = [P, I32, P, P]
    lib.lbm_bench_copy.argtypes = [P, P, SZ, P]
    lib.lbm_bench_copy_cached.argtypes = [P, P, SZ, P]
    lib.lbm_set_diffusion.argtypes = [P, I32, P]
    lib.lbm_adjoint_segment.argtypes = [P, I32, P, I32, P, P, P]
    lib.lbm_free.argtypes = [P]
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_abi_version.argtypes = []
    for name in EXPORTS:
        if name not in ("lbm_last_error",):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(status: int) -> int:
    if status != LBM_OK:
        raise LbmError(status, lib().lbm_last_error().decode())
    return status


def _dptr(t: Optional[torch.Tensor], dtype=torch.float64) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor, got {t.dtype} on {t.device}")
    return t.data_ptr()


def _ptr_array(ts: Optional[Sequence[Optional[torch.Tensor]]]):
    if ts is None:
        return None
    arr = (ctypes.c_void_p * len(ts))(*[_dptr(t) for t in ts])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), arr


def make_params(nx, ny, dx, dt, lam, D_const=0.0, mode="f64", aux=LBM_AUX_LOCAL, scale_log2=15,
                phi_ref=0.0, boundary=LBM_BC_PERIODIC, tau3=0.0, nz=0, lattice=None, round_seed=0) -> lbm_params:
    """nz >= 3 selects a 3D lattice (nx * ny * nz nodes): D3Q19 unless lattice says D3Q27 (19 or 27
    are accepted for the LBM_LATTICE_* values); nz = 0 is D2Q9.  round_seed: seed of the rounding
    stream of mode "f16sr"."""
    store, math = MODES[mode]
    if lattice is None:
        lattice = LBM_LATTICE_D3Q19 if nz else LBM_LATTICE_D2Q9
    else:
        lattice = {9: LBM_LATTICE_D2Q9, 19: LBM_LATTICE_D3Q19, 27: LBM_LATTICE_D3Q27}.get(int(lattice), int(lattice))
    return lbm_params(int(nx), int(ny), float(dx), float(dt), float(lam), float(D_const), store, math, int(aux),
                      int(scale_log2), float(phi_ref), int(boundary), int(round_seed), float(tau3), lattice, int(nz))


def lbm_abi_version() -> int:
    return lib().lbm_abi_version()


def lbm_last_error() -> str:
    return lib().lbm_last_error().decode()


def lbm_workspace_size(params: Sequence[lbm_params]) -> int:
    arr = (lbm_params * len(params))(*params)
    out = ctypes.c_size_t()
    _check(lib().lbm_workspace_size(len(params), arr, ctypes.byref(out)))
    return out.value


def lbm_init(params: Sequence[lbm_params], fields: Sequence[dict], workspace: Optional[torch.Tensor] = None,
             stream: Optional[torch.cuda.Stream] = None) -> ctypes.c_void_p:
    """fields[k]: dict with device FP64 tensors phi0, ux, uy, optional D, and uz on 3D lattices (each
    [ny, nx], 3D [nz, ny, nx])."""
    n = len(params)
    parr = (lbm_params * n)(*params)
    farr = (lbm_fields * n)(*[lbm_fields(_dptr(f["phi0"]), _dptr(f["ux"]), _dptr(f["uy"]), _dptr(f.get("D")),
                                         _dptr(f.get("uz"))) for f in fields])
    ws_ptr = None if workspace is None else workspace.data_ptr()
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    s = (stream or torch.cuda.current_stream()).cuda_stream
    ctx = ctypes.c_void_p()
    _check(lib().lbm_init(ctypes.byref(ctx), n, parr, farr, ws_ptr, ws_bytes, s))
    return ctx


def lbm_step(ctx, nsteps: int, ux=None, uy=None, S=None, dSdt=None) -> None:
    pu, pv, ps, pd = (_ptr_array(a) for a in (ux, uy, S, dSdt))
    _check(lib().lbm_step(ctx, int(nsteps), pu[0] if pu else None, pv[0] if pv else None, ps[0] if ps else None,
                          pd[0] if pd else None))


def lbm_set_velocity(ctx, inst: int, ux: torch.Tensor, uy: torch.Tensor, uz: Optional[torch.Tensor] = None) -> None:
    _check(lib().lbm_set_velocity(ctx, int(inst), _dptr(ux), _dptr(uy), _dptr(uz)))


def lbm_set_diffusion(ctx, inst: int, D: torch.Tensor) -> None:
    _check(lib().lbm_set_diffusion(ctx, int(inst), _dptr(D)))


def lbm_set_dirichlet(ctx, inst: int, phi_b: torch.Tensor) -> None:
    _check(lib().lbm_set_dirichlet(ctx, int(inst), _dptr(phi_b)))


def lbm_macros(ctx, inst: int = 0, phi_out: Optional[torch.Tensor] = None, ref: Optional[torch.Tensor] = None,
               raise_nonfinite: bool = True) -> dict:
    st = lbm_stats()
    rc = lib().lbm_macros(ctx, int(inst), _dptr(phi_out), _dptr(ref), ctypes.byref(st))
    if rc != LBM_OK and not (rc == LBM_E_NONFINITE and not raise_nonfinite):
        _check(rc)
    d = st.as_dict()
    d["status"] = rc
    return d


def lbm_macros_static(ctx, inst: int = 0, phi_out: Optional[torch.Tensor] = None, ref: Optional[torch.Tensor] = None,
                      raise_nonfinite: bool = True) -> dict:
    st = lbm_stats()
    rc = lib().lbm_macros_static(ctx, int(inst), _dptr(phi_out), _dptr(ref), ctypes.byref(st))
    if rc != LBM_OK and not (rc == LBM_E_NONFINITE and not raise_nonfinite):
        _check(rc)
    d = st.as_dict()
    d["status"] = rc
    return d


def lbm_populations(ctx, inst: int, out: torch.Tensor) -> None:
    _check(lib().lbm_populations(ctx, int(inst), _dptr(out)))


def lbm_state_bytes(ctx, inst: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().lbm_state_bytes(ctx, int(inst), ctypes.byref(out)))
    return out.value


def lbm_state_save(ctx, inst: int, dst: torch.Tensor) -> None:
    _check(lib().lbm_state_save(ctx, int(inst), _dptr(dst, dst.dtype)))


def lbm_state_load(ctx, inst: int, src: torch.Tensor, step: int) -> None:
    _check(lib().lbm_state_load(ctx, int(inst), _dptr(src, src.dtype), int(step)))


def lbm_set_launch(ctx, inst: int, rows: int, xcd_remap: int = 1, tile_width: int = 64, max_waves: int = 0,
                   xcd_rows: int = 0, stores: int = 0, fuse: int = 1) -> None:
    cfg = lbm_launch(int(rows), int(xcd_remap), int(tile_width), int(max_waves), int(xcd_rows), int(stores),
                     int(fuse))
    _check(lib().lbm_set_launch(ctx, int(inst), ctypes.byref(cfg)))


def lbm_get_launch(ctx, inst: int = 0) -> dict:
    cfg = lbm_launch()
    _check(lib().lbm_get_launch(ctx, int(inst), ctypes.byref(cfg)))
    return {"rows": cfg.rows, "xcd_remap": cfg.xcd_remap, "tile_width": cfg.tile_width, "max_waves": cfg.max_waves,
            "xcd_rows": cfg.xcd_rows, "stores": cfg.stores, "fuse": cfg.fuse}


def lbm_set_batch(ctx, policy: int, blocks: int = 0, max_waves: int = 0) -> None:
    cfg = lbm_batch(int(policy), int(blocks), int(max_waves))
    _check(lib().lbm_set_batch(ctx, ctypes.byref(cfg)))


def lbm_get_batch(ctx) -> dict:
    cfg = lbm_batch()
    _check(lib().lbm_get_batch(ctx, ctypes.byref(cfg)))
    return {"policy": cfg.policy, "blocks": cfg.blocks, "max_waves": cfg.max_waves}


def lbm_adjoint_bytes(ctx, inst: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().lbm_adjoint_bytes(ctx, int(inst), ctypes.byref(out)))
    return out.value


def lbm_adjoint_seed(ctx, inst: int, dLdphi: torch.Tensor, lam: torch.Tensor) -> None:
    _check(lib().lbm_adjoint_seed(ctx, int(inst), _dptr(dLdphi), _dptr(lam, lam.dtype)))


def lbm_adjoint_step(ctx, inst: int, state: torch.Tensor, lam_in: torch.Tensor, lam_out: torch.Tensor,
                     dLdD: torch.Tensor) -> None:
    _check(lib().lbm_adjoint_step(ctx, int(inst), _dptr(state, state.dtype), _dptr(lam_in, lam_in.dtype),
                                  _dptr(lam_out, lam_out.dtype), _dptr(dLdD)))


def lbm_adjoint_segment(ctx, inst: int, states: torch.Tensor, nsteps: int, lam: torch.Tensor, lam_tmp: torch.Tensor,
                        dLdD: torch.Tensor) -> None:
    _check(lib().lbm_adjoint_segment(ctx, int(inst), _dptr(states, states.dtype), int(nsteps), _dptr(lam, lam.dtype),
                                     _dptr(lam_tmp, lam_tmp.dtype), _dptr(dLdD)))


def lbm_adjoint_init(ctx, inst: int, lam0: torch.Tensor, dLdphi0: torch.Tensor) -> None:
    _check(lib().lbm_adjoint_init(ctx, int(inst), _dptr(lam0, lam0.dtype), _dptr(dLdphi0)))


def lbm_bench_copy(dst: torch.Tensor, src: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> None:
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("dst smaller than src")
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib().lbm_bench_copy(dst.data_ptr(), src.data_ptr(), n, s))


def lbm_bench_copy_cached(dst: torch.Tensor, src: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> None:
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("dst smaller than src")
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib().lbm_bench_copy_cached(dst.data_ptr(), src.data_ptr(), n, s))


def lbm_free(ctx) -> None:
    _check(lib().lbm_free(ctx))
