"""Mutation check of the oracle pins (CPU only).

Each case plants one plausible mistake in a private copy of the oracle's C source (a dropped term,
a wrong sign, factor or index, a transposed operand, a reversed streaming direction), builds that
copy, and runs the pin suite against it in a subprocess.  Every mutant must fail at least one pin.
The repository's oracle is never modified.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
PINS_3D = os.path.join(ROOT, "tests", "test_oracle_pins_3d.py")

MUTANTS = [
    ("drop third-order equilibrium", "+ s3 / (6.0 * cs2 * cs2 * cs2)", ""),
    ("equilibrium second-order factor", "s2 / (2.0 * cs2 * cs2)", "s2 / (cs2 * cs2)"),
    ("Hermite H2 without delta", "- cs2 * kd(a, b);\n}", ";\n}"),
    ("Hermite H3 index", "ecomp(i, b, c) * kd(g, a)", "ecomp(i, b, c) * kd(a, b)"),
    ("velocity sign", "{0, 0, 1, 0, -1, 1, 1, -1, -1}", "{0, 0, 1, 0, -1, -1, 1, -1, -1}"),
    ("omega1 factor", "(1.0 - 1.0 / tau1) * W[i] * r1", "(1.0 - 0.5 / tau1) * W[i] * r1"),
    ("omega2 from tau1", "(1.0 - 1.0 / tau2) * W[i] * r2", "(1.0 - 1.0 / tau1) * W[i] * r2"),
    ("second-order neq factor", "* r2 / (2.0 * cs2 * cs2)", "* r2 / (cs2 * cs2)"),
    ("tau1 from kappa", "*tau1 = 0.5 + kappa / (cs2 * dt);", "*tau1 = 0.5 + 2.0 * kappa / (cs2 * dt);"),
    ("tau2 from Lambda", "*tau2 = 0.5 + lambda / (*tau1 - 0.5);", "*tau2 = 0.5 + lambda * (*tau1 - 0.5);"),
    ("beta", "real beta = 1.0 - 1.0 / (2.0 * tau1);", "real beta = 1.0 - 1.0 / tau1;"),
    ("aux sign", "real G = W[i] * eA / cs2 * beta;", "real G = -W[i] * eA / cs2 * beta;"),
    ("aux transposed gradient", "u[a][hi[b]] - u[a][lo[b]]", "u[b][hi[a]] - u[b][lo[a]]"),
    ("aux without phi", "A[a] = phi * s;", "A[a] = s;"),
    ("aux difference spacing", "double h[2] = {2.0 * dx, 2.0 * dx};", "double h[2] = {dx, dx};"),
    ("one-sided edge spacing", "if (x == 0) { lo[0] = n; h[0] = dx; }", "if (x == 0) { lo[0] = n; h[0] = 2.0 * dx; }"),
    ("one-sided edge side", "else if (y == ny - 1) { hi[1] = n; h[1] = dx; }",
     "else if (y == ny - 1) { lo[1] = n; h[1] = dx; }"),
    ("anti-bounce-back sign", "g_out[o * N + n] = -P + (geq_w[i] + geq_w[o]);", "g_out[o * N + n] = P + (geq_w[i] + geq_w[o]);"),
    ("anti-bounce-back odd part", "-P + (geq_w[i] + geq_w[o])", "-P + 2.0 * geq_w[i]"),
    ("walls keep the wrapped derivative", "if (p->boundary == 1 || p->boundary == 2) {", "if (p->boundary == 1) {"),
    ("MRT third-order rate", "(1.0 - 1.0 / tau3) * W[i] * r3", "(1.0 - 1.0 / tau2) * W[i] * r3"),
    ("MRT third-order factor", "r3 / (6.0 * cs2 * cs2 * cs2)", "r3 / (2.0 * cs2 * cs2 * cs2)"),
    ("NEE sign", "geq_b[i] + (g[i * N + f] - geq_f[i])", "geq_b[i] - (g[i * N + f] - geq_f[i])"),
    ("NEE neighbour row", "yf = y + (y == 0) - (y == ny - 1);", "yf = y + (y == 0);"),
    ("NEE equilibrium velocity", "ORC(equilibrium)(phi_b[b], ux[b], uy[b], c, geq_b);",
     "ORC(equilibrium)(phi_b[b], ux[f], uy[f], c, geq_b);"),
    ("aux neighbour", "nb[1][0] = (size_t)wrap(y - 1, ny) * nx + x;", "nb[1][0] = (size_t)wrap(y + 1, ny) * nx + x;"),
    ("aux without dt", "real P = C[i] + dt * G +", "real P = C[i] + G +"),
    ("flux-form sign", "s += dflux - un[a] * dmass;", "s += dflux + un[a] * dmass;"),
    ("flux-form index", "real dmass = (phi_all[q] * u[b][q] - phi_all[m] * u[b][m])",
     "real dmass = (phi_all[q] * u[a][q] - phi_all[m] * u[a][m])"),
    ("source zeroth order", "real F = W[i] * src +", "real F ="),
    ("source without beta", "+ beta * W[i] * eu / cs2 * src", "+ W[i] * eu / cs2 * src"),
    ("source derivative half", "0.5 * dt * dt * dF", "dt * dt * dF"),
    ("source derivative operand", "beta * W[i] * eu / cs2 * dsrc;", "beta * W[i] * eu / cs2 * src;"),
    ("streaming direction", "wrap(ty, ny) * nx + wrap(x + EX[i], nx)",
     "wrap(y - EY[i], ny) * nx + wrap(x - EX[i], nx)"),
]

MUTANTS_3D = [
    ("z velocity table", "static const int EZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,",
     "static const int EZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1,"),
    ("edge weight", "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};",
     "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 18.0};"),
    ("drop third-order equilibrium", "+ s3 / (6.0 * cs2 * cs2 * cs2)", ""),
    ("tau2 from tau1", "(1.0 - 1.0 / tau2) * W[i] * r2", "(1.0 - 1.0 / tau1) * W[i] * r2"),
    ("z difference neighbour", "lo[2] = ((size_t)wrap(z - 1, nz) * ny + y) * nx + x;",
     "lo[2] = ((size_t)wrap(z + 1, nz) * ny + y) * nx + x;"),
    ("aux without phi", "A[a] = phi * s;", "A[a] = s;"),
    ("source without beta", "+ beta * W[i] * eu / cs2 * src;", "+ W[i] * eu / cs2 * src;"),
    ("z streaming direction", "wrap(z + EZ[i], nz)", "wrap(z - EZ[i], nz)"),
    ("tau1 from kappa", "const double tau1 = 0.5 + kappa / (cs2 * dt);", "const double tau1 = 0.5 + 2.0 * kappa / (cs2 * dt);"),
    ("velocity components swapped", "const double un[3] = {u[n], u[N + n], u[2 * N + n]};",
     "const double un[3] = {u[n], u[2 * N + n], u[N + n]};"),
    # D3Q27 only
    ("D3Q27 corner x table", "1, -1, 1, -1, 1, -1, -1, 1};", "1, -1, 1, -1, -1, 1, -1, 1};"),
    ("D3Q27 corner z table", "1, -1, -1, 1, 1, -1, 1, -1};", "1, -1, 1, -1, 1, -1, 1, -1};"),
    ("D3Q27 face weight", "2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,",
     "2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 1.0 / 18.0,"),
    ("D3Q27 corner weight", "1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};",
     "1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 108.0};"),
    ("D3Q27 edge and corner weights exchanged",
     "1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,\n                               1.0 / 216.0",
     "1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 216.0,\n                               1.0 / 54.0"),
]

# the diagnostics written out in the oracle's Python layer
MUTANTS_PY = [
    ("L2 error without square root", "return math.sqrt(math.fsum((d * d).tolist()) / math.fsum((r * r).tolist()))",
     "return math.fsum((d * d).tolist()) / math.fsum((r * r).tolist())"),
    ("L2 error normalised by the numerical field", "r = np.asarray(phi_ref, np.float64).ravel()",
     "r = np.asarray(phi_num, np.float64).ravel()"),
    ("max error without absolute value",
     "return float(np.max(np.abs(np.asarray(phi_num, np.float64) - np.asarray(phi_ref, np.float64))))",
     "return float(np.max(np.asarray(phi_num, np.float64) - np.asarray(phi_ref, np.float64)))"),
    ("RMS error node count", "return math.sqrt(math.fsum((d * d).tolist()) / d.size)",
     "return math.sqrt(math.fsum((d * d).tolist()) / (d.size - 1))"),
    ("mass by a plain float sum", "return math.fsum(np.asarray(phi_field, dtype=np.float64).ravel().tolist())",
     "return float(np.asarray(phi_field, dtype=np.float64).ravel().sum())"),
]

# Mistakes in the FP16 storage codes (oracle/rounding.py), checked against their own pins.
PINS_SR = os.path.join(ROOT, "tests", "test_oracle_pins_sr.py")
MUTANTS_SR = [
    ("stochastic rounding comparison inclusive", "up = np.asarray(r, dtype=np.float64) < m",
     "up = np.asarray(r, dtype=np.float64) <= m"),
    ("rounding up for the large integers", "up = np.asarray(r, dtype=np.float64) < m",
     "up = np.asarray(r, dtype=np.float64) >= 2 ** RBITS - m"),
    ("finer bits rounded up", "m = np.floor((a - lo) / ulp * 2 ** RBITS)", "m = np.ceil((a - lo) / ulp * 2 ** RBITS)"),
    ("twelve random bits per value", "RBITS = 13  #", "RBITS = 12  #"),
    ("SplitMix64 increment", "GAMMA = 0x9E3779B97F4A7C15", "GAMMA = 0x9E3779B97F4A7C13"),
    ("SplitMix64 first shift", "z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64",
     "z = ((z ^ (z >> 31)) * 0xBF58476D1CE4E5B9) & MASK64"),
    ("SplitMix64 array shift", "z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)",
     "z = (z ^ (z >> np.uint64(28))) * np.uint64(0x94D049BB133111EB)"),
    ("stream output counted from 1", "(k + np.uint64(1)) * np.uint64(GAMMA)", "k * np.uint64(GAMMA)"),
    ("one output per node", "first = 2 * (level.astype(np.uint64)", "first = (level.astype(np.uint64)"),
    ("straddling field halves swapped", "v = (lo >> np.uint64(b)) | (hi << np.uint64(64 - b))",
     "v = (hi >> np.uint64(b - 64 + 13)) | (lo << np.uint64(64 - b))"),
    ("nearest instead of lower neighbour", "h = np.where(h.astype(np.float64) > a, np.nextafter(h, np.float16(0)), h)",
     "h = h"),
    ("sign dropped", "return np.where(np.signbit(v), -out, out)", "return out"),
    ("shift after scaling", "return ((g32 - w32) * np.float32(2.0 ** scale_log2)).astype(np.float32)",
     "return (g32 * np.float32(2.0 ** scale_log2) - w32).astype(np.float32)"),
]

_PLUGIN = '''
import importlib.util, os, sys
spec = importlib.util.spec_from_file_location("oracle", os.environ["MUTANT_ORACLE"])
mod = importlib.util.module_from_spec(spec)
sys.modules["oracle"] = mod
spec.loader.exec_module(mod)
'''


def _run_mutant(name, old, new, tmp_path, source, pins):
    with open(os.path.join(ROOT, "oracle", source)) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"mutation site for '{name}' must be unique"
    mdir = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), mdir,
                    ignore=shutil.ignore_patterns("*.so", "*.o", "__pycache__"))
    (mdir / source).write_text(src.replace(old, new))
    (tmp_path / "mutant_plugin.py").write_text(_PLUGIN)
    env = dict(os.environ, MUTANT_ORACLE=str(mdir / "__init__.py"), PYTHONPATH=str(tmp_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "mutant_plugin", "-p", "no:cacheprovider",
                        pins], cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"mutant '{name}' survived the pins:\n{r.stdout[-2000:]}"
    assert "FAILED" in r.stdout


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    _run_mutant(name, old, new, tmp_path, "lbm_oracle.c", PINS)


@pytest.mark.parametrize("name,old,new", MUTANTS_3D, ids=[m[0] for m in MUTANTS_3D])
def test_3d_mutant_is_caught(name, old, new, tmp_path):
    _run_mutant(name, old, new, tmp_path, "lbm_oracle_3d.c", PINS_3D)


@pytest.mark.parametrize("name,old,new", MUTANTS_PY, ids=[m[0] for m in MUTANTS_PY])
def test_diagnostics_mutant_is_caught(name, old, new, tmp_path):
    _run_mutant(name, old, new, tmp_path, "__init__.py", PINS)


@pytest.mark.parametrize("name,old,new", MUTANTS_SR, ids=[m[0] for m in MUTANTS_SR])
def test_rounding_mutant_is_caught(name, old, new, tmp_path):
    _run_mutant(name, old, new, tmp_path, "rounding.py", PINS_SR)
