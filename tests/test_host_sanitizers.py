"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU, no GPU).

- The oracle: tests/sanitize/oracle2d_driver.c and oracle3d_driver.c include the oracle's C sources, so
  the whole oracle is built with both sanitizers (gcc, -fno-sanitize-recover: the first finding aborts
  the run).  The drivers run jobs covering every aux form, boundary, MRT-R, D fields, sources and both
  3D lattices, and their results must equal the regular oracle build's bit for bit.
- The library: its host code (argument validation, workspace sizes, pitches, error messages, NULL
  contexts; everything that runs before a device call) is built with both sanitizers on the host side
  only and driven by tests/sanitize/api_driver.c, with leak detection on.
"""
import hashlib
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _gcc_driver(tmp_path, name):
    exe = str(tmp_path / name)
    src = os.path.join(HERE, "sanitize", name + ".c")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", *SAN, src, "-o", exe,
                    "-lm"], check=True)
    return exe


def _run(exe, jobs, tmp_path):
    jf, of = str(tmp_path / "jobs.bin"), str(tmp_path / "out.bin")
    with open(jf, "wb") as f:
        f.write(jobs)
    r = subprocess.run([exe, jf, of], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return np.fromfile(of, dtype=np.float64)


def test_oracle_2d_under_sanitizers(tmp_path):
    rng = np.random.default_rng(20231216)
    nx, ny = 13, 11
    dx = 1.0 / nx
    dt = dx / 10.0
    sh = (ny, nx)
    phi0 = 1.0 + 0.1 * rng.random(sh)
    ux, uy = rng.uniform(-0.5, 0.5, sh), rng.uniform(-0.5, 0.5, sh)
    D = 1e-3 * (1.0 + 0.5 * rng.random(sh))
    S, dSdt = 1e-2 * rng.standard_normal(sh), 1e-2 * rng.standard_normal(sh)
    phib = 1.0 + 0.05 * rng.random(sh)
    cases = [  # aux, boundary, tau3, steps, D, S, dSdt, phi_b
        (oracle.AUX_LOCAL, oracle.BC_PERIODIC, 0.0, 4, None, None, None, None),
        (oracle.AUX_FLUX, oracle.BC_PERIODIC, 0.0, 4, D, None, None, None),
        (oracle.AUX_NONE, oracle.BC_PERIODIC, 0.0, 3, None, S, dSdt, None),
        (oracle.AUX_LOCAL, oracle.BC_NEE, 0.0, 3, D, None, None, phib),
        (oracle.AUX_LOCAL, oracle.BC_WALLS, 0.0, 3, None, S, None, phib),
        (oracle.AUX_LOCAL, oracle.BC_PERIODIC, 0.7, 3, D, None, None, None),
    ]
    jobs, want = b"", []
    for aux, bc, tau3, steps, Df, Sf, dSf, pb in cases:
        p = oracle.Problem(nx, ny, dx, dt, 0.25, 1e-3, aux, bc, tau3)
        g0 = oracle.init(p, phi0, ux, uy)
        want.append(oracle.run(p, g0, steps, ux, uy, Df, Sf, dSf, pb).ravel())
        head = np.array([nx, ny, aux, bc, steps, Df is not None, Sf is not None, dSf is not None, pb is not None],
                        dtype=np.int32)
        jobs += head.tobytes() + np.array([dx, dt, 0.25, 1e-3, tau3]).tobytes()
        for a in (g0, ux, uy, Df, Sf, dSf, pb):
            if a is not None:
                jobs += np.ascontiguousarray(a, dtype=np.float64).tobytes()
    got = _run(_gcc_driver(tmp_path, "oracle2d_driver"), jobs, tmp_path)
    assert np.array_equal(got, np.concatenate(want))


def test_oracle_3d_under_sanitizers(tmp_path):
    rng = np.random.default_rng(20231217)
    jobs, want = b"", []
    for q, aux, with_D in ((19, oracle.AUX_LOCAL, False), (27, oracle.AUX_LOCAL, True), (19, oracle.AUX_NONE, True)):
        nx, ny, nz = 5, 4, 3
        dx = 1.0 / nx
        dt = dx / 10.0
        p = oracle.Problem3(nx, ny, nz, dx, dt, 0.25, 1e-3, aux, q)
        phi0 = 1.0 + 0.1 * rng.random(p.shape)
        u = rng.uniform(-0.5, 0.5, (3,) + p.shape)
        D = 1e-3 * (1.0 + 0.5 * rng.random(p.shape)) if with_D else None
        g0 = oracle.init3(p, phi0, u)
        want.append(oracle.run3(p, g0, 3, u, D).ravel())
        jobs += np.array([nx, ny, nz, aux, q, 3, with_D], dtype=np.int32).tobytes()
        jobs += np.array([dx, dt, 0.25, 1e-3]).tobytes() + g0.tobytes() + np.ascontiguousarray(u).tobytes()
        if with_D:
            jobs += D.tobytes()
    got = _run(_gcc_driver(tmp_path, "oracle3d_driver"), jobs, tmp_path)
    assert np.array_equal(got, np.concatenate(want))


LIB_SOURCES = ["lbm_kernels.hip", "lbm_kernels3d.hip", "lbm_fused.hip", "lbm_adjoint.hip", "lbm_api.hip"]
CSRC = os.path.join(ROOT, "paper_2312_10316_amd", "csrc")


def _sanitized_library_objects():
    """The library's objects with the host side built under both sanitizers (device code as usual),
    cached by a hash of the sources under the temp directory (a full build takes about a minute)."""
    if shutil.which("/opt/rocm/bin/hipcc") is None:
        pytest.skip("hipcc not found")
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + f.read())
    out = os.path.join(tempfile.gettempdir(), f"lbm_host_sanitize_{h.hexdigest()[:16]}")
    objs = [os.path.join(out, s.replace(".hip", ".o")) for s in LIB_SOURCES]
    if all(os.path.exists(o) for o in objs):
        return objs
    os.makedirs(out, exist_ok=True)
    flags = ["-std=c++17", "-O1", "-fPIC", "--offload-arch=gfx950", "-fno-gpu-rdc",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-g"):
        flags += ["-Xarch_host", f]  # host code only
    procs = []
    for s, o in zip(LIB_SOURCES, objs):
        procs.append(subprocess.Popen(["/opt/rocm/bin/hipcc", *flags, "-c", os.path.join(CSRC, s), "-o", o + ".tmp"],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL))
    assert all(p.wait() == 0 for p in procs), "sanitized host build of the library failed"
    for o in objs:
        os.replace(o + ".tmp", o)
    return objs


def test_library_host_code_under_sanitizers(tmp_path):
    objs = _sanitized_library_objects()
    clang = "/opt/rocm/llvm/bin/clang"
    drv = str(tmp_path / "api_driver.o")
    subprocess.run([clang, "-std=c11", "-O1", "-g", *SAN, "-c", os.path.join(HERE, "sanitize", "api_driver.c"),
                    "-o", drv], check=True)
    exe = str(tmp_path / "api_driver")
    subprocess.run([clang + "++", *SAN, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                    "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    last = r.stdout.strip().splitlines()[-1]
    assert last.startswith("ok ") and int(last.split()[1]) > 100, last
