"""The C-ABI library loads and exports what include/lbm.h declares; host-side validation (CPU only,
no HIP compute call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2312_10316_amd import lbm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(lbm_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lbm_init", "lbm_step", "lbm_macros", "lbm_free"):
        assert required in names
    assert set(names) == set(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (lbm_\w+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported
    assert L.lbm_abi_version() == 9


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lbm_params), '
                    'offsetof(lbm_params, phi_ref), offsetof(lbm_params, store), sizeof(lbm_fields), '
                    'sizeof(lbm_stats), offsetof(lbm_stats, nonfinite), sizeof(lbm_launch), '
                    'offsetof(lbm_launch, xcd_rows), sizeof(lbm_batch)); return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{os.path.dirname(HEADER)}", str(prog), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(L.lbm_params), L.lbm_params.phi_ref.offset, L.lbm_params.store.offset,
                    ctypes.sizeof(L.lbm_fields), ctypes.sizeof(L.lbm_stats), L.lbm_stats.nonfinite.offset,
                    ctypes.sizeof(L.lbm_launch), L.lbm_launch.xcd_rows.offset, ctypes.sizeof(L.lbm_batch)]


def _p(**kw):
    base = dict(nx=64, ny=64, dx=1 / 32, dt=1 / 320, lam=0.25, D_const=1e-3, mode="f64")
    base.update(kw)
    return L.make_params(**base)


def test_workspace_size_scales_with_storage():
    b64 = L.lbm_workspace_size([_p(nx=1024, ny=1024)])
    b32 = L.lbm_workspace_size([_p(nx=1024, ny=1024, mode="f32")])
    b16 = L.lbm_workspace_size([_p(nx=1024, ny=1024, mode="f16s")])
    assert b64 > b32 > b16 > 2 * 9 * 1024 * 1024 * 2
    assert L.lbm_workspace_size([_p(), _p(nx=100, ny=37)]) > L.lbm_workspace_size([_p()])


@pytest.mark.parametrize("mode,esize", [("f64", 8), ("f32", 4), ("f16s", 2)])
def test_pitch_rule(mode, esize):
    """Host-only layout query: nx rounded up to 64 elements, plus 64 when the rounded row segment
    would span a multiple of 4 KiB (the population rows of every width avoid 4 KiB strides)."""
    for nx in (3, 63, 64, 65, 100, 512, 1000, 1024, 2048, 2049, 3072, 4096, 8192):
        pitch = L.pitch_of(_p(nx=nx, ny=5, mode=mode))
        assert pitch >= nx and pitch % 64 == 0 and pitch - nx < 128
        assert (pitch * esize) % 4096 != 0
        base = (nx + 63) // 64 * 64
        assert pitch == base or (base * esize) % 4096 == 0
    with pytest.raises(L.LbmError):
        L.pitch_of(_p(nx=2))


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=2), "must be >= 3"),
    (dict(ny=0), "must be >= 3"),
    (dict(dx=0.0), "dx and dt"),
    (dict(dt=float("nan")), "dx and dt"),
    (dict(lam=-1.0), "lambda"),
    (dict(scale_log2=40, mode="f16s"), "scale_log2"),
])
def test_invalid_parameters_are_rejected(kw, msg):
    with pytest.raises(L.LbmError) as ei:
        L.lbm_workspace_size([_p(**kw)])
    assert ei.value.status == L.LBM_E_ARG
    assert msg in str(ei.value)


def test_maximum_sizes():
    """2^31 nodes is the largest instance (D2Q9 and D3Q19); one more node is rejected; the
    workspace of the largest FP16 instance is its 2 x 9 x 2 bytes per node plus fields."""
    big = _p(nx=65536, ny=32768, mode="f16s")  # 2^31 nodes
    ws = L.lbm_workspace_size([big])
    assert ws > 2 * 9 * 2 * (1 << 31)
    with pytest.raises(L.LbmError, match="2\\^31"):
        L.lbm_workspace_size([_p(nx=65536, ny=32769)])
    L.lbm_workspace_size([_p(nx=1 << 24, ny=3)])  # the longest row
    L.lbm_workspace_size([_p(nx=1 << 24, ny=3, nz=3)])
    with pytest.raises(L.LbmError, match="2\\^24"):
        L.lbm_workspace_size([_p(nx=(1 << 24) + 1, ny=3)])
    assert L.lbm_workspace_size([_p(nx=1024, ny=1024, nz=2048)]) > 2 * 19 * 8 * (1 << 31)
    with pytest.raises(L.LbmError, match="2\\^31"):
        L.lbm_workspace_size([_p(nx=1024, ny=1024, nz=2049)])


@pytest.mark.parametrize("kw,msg", [
    (dict(nz=2), "must be >= 3"),
    (dict(nz=-5), "must be >= 3"),
    (dict(nz=2, lattice=27), "must be >= 3"),
    (dict(nz=8, lattice=3), "unknown lattice"),
    (dict(nz=8, lattice=-1), "unknown lattice"),
])
def test_invalid_3d_parameters(kw, msg):
    with pytest.raises(L.LbmError) as ei:
        L.lbm_workspace_size([_p(**kw)])
    assert ei.value.status == L.LBM_E_ARG
    assert msg in str(ei.value)


@pytest.mark.parametrize("q", [19, 27])
def test_3d_unsupported_combinations(q):
    for kw in (dict(aux=L.LBM_AUX_FLUX), dict(boundary=L.LBM_BC_NEE), dict(tau3=0.9)):
        with pytest.raises(L.LbmError) as ei:
            L.lbm_workspace_size([_p(nz=8, lattice=q, **kw)])
        assert ei.value.status == L.LBM_E_UNSUPPORTED, kw


def test_d3q27_workspace_holds_27_planes():
    """Two population buffers of 27 planes (plus the same fields as D3Q19): the difference to a
    D3Q19 instance of the same size is exactly 2 x 8 planes of the storage type."""
    for mode, elem in (("f64", 8), ("f32", 4)):
        a = L.lbm_workspace_size([_p(nx=100, ny=20, nz=10, mode=mode, lattice=19)])
        b = L.lbm_workspace_size([_p(nx=100, ny=20, nz=10, mode=mode, lattice=27)])
        pitch = L.pitch_of(_p(nx=100, ny=20, nz=10, mode=mode, lattice=27))
        assert b - a >= 2 * 8 * 20 * 10 * pitch * elem
        assert b - a <= 2 * 8 * 20 * 10 * pitch * elem + 4096


def test_fp64_math_needs_fp64_storage():
    p = _p(mode="f32")
    p.math = L.LBM_MATH_F64
    with pytest.raises(L.LbmError, match="FP64 math needs FP64 storage"):
        L.lbm_workspace_size([p])


def test_null_context_calls_fail_cleanly():
    lib = L.lib()
    assert lib.lbm_free(None) == L.LBM_OK
    assert lib.lbm_step(None, 1, None, None, None, None) == L.LBM_E_STATE
    st = L.lbm_stats()
    assert lib.lbm_macros(None, 0, None, None, ctypes.byref(st)) == L.LBM_E_STATE
    assert "bad context" in L.lbm_last_error()
    assert lib.lbm_init(None, 1, None, None, None, 0, None) == L.LBM_E_ARG
    assert lib.lbm_set_diffusion(None, 0, None) == L.LBM_E_STATE
    assert lib.lbm_adjoint_segment(None, 0, None, 1, None, None, None) == L.LBM_E_STATE
    assert lib.lbm_bench_copy_cached(None, None, 16, None) == L.LBM_E_ARG
    assert lib.lbm_bench_copy_cached(16, 16, 8, None) == L.LBM_E_ARG  # bytes not a multiple of 16
