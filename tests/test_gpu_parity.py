"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle, on the same seeded inputs.

FP64 storage + FP64 math must match the oracle to 1e-12 in the normalised max-abs sense
(max |g_gpu - g_orc| / max |g_orc| over all nine population planes).  Reduced-precision modes are
held to bounds derived from their rounding units (documented with each test).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2312_10316_amd import Solver, lbm

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def smooth_field(nx, ny, seed, lo, hi):
    """Seeded smooth periodic field in [lo, hi] (a few random Fourier modes)."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx) * 2 * np.pi / nx
    y = np.arange(ny) * 2 * np.pi / ny
    Y, X = np.meshgrid(y, x, indexing="ij")
    f = np.zeros((ny, nx))
    for _ in range(4):
        kx, ky = rng.integers(0, 3, 2)
        f += rng.uniform(-1, 1) * np.cos(kx * X + ky * Y + rng.uniform(0, 2 * np.pi))
    f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
    return lo + (hi - lo) * f


def case_fields(nx, ny, seed, U=0.3, D0=2e-3, varD=True):
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    rng = np.random.default_rng(seed)
    c = 4.0
    ux = c * (U * smooth_field(nx, ny, seed + 1, -1, 1))
    uy = c * (U * smooth_field(nx, ny, seed + 2, -1, 1))
    phi0 = 0.2 + smooth_field(nx, ny, seed + 3, 0, 1) + 0.05 * rng.uniform(0, 1, (ny, nx))
    D = D0 * smooth_field(nx, ny, seed + 4, 0.5, 1.5) if varD else None
    return dict(dx=dx, dt=dx / c, ux=ux, uy=uy, phi0=phi0, D=D, D_const=D0)


def run_pair(nx, ny, f, steps, aux, lam=0.25, mode="f64", sources=None):
    """Runs the GPU path and the oracle from g = g_eq(phi0, u); returns (g_gpu, g_orc, stats)."""
    p = lbm.make_params(nx, ny, f["dx"], f["dt"], lam, f["D_const"], mode, aux)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy")}
    if f["D"] is not None:
        fields["D"] = dev(f["D"])
    s = Solver([(p, fields)])
    op = O.Problem(nx, ny, f["dx"], f["dt"], lam, f["D_const"], aux)
    g = O.init(op, f["phi0"], f["ux"], f["uy"])
    if sources is None:
        s.step(steps)
        g = O.run(op, g, steps, f["ux"], f["uy"], f["D"])
    else:
        for t in range(steps):
            S, dS = sources(t)
            s.step(1, S=[dev(S)], dSdt=[dev(dS)])
            g = O.step(op, g, f["ux"], f["uy"], f["D"], S, dS)
    g_gpu = s.populations().cpu().numpy()
    st = s.macros()
    s.close()
    return g_gpu, g, st


# ---- FP64 parity ---------------------------------------------------------------------------------

def test_fp64_rotating_pulse_64():
    """The 64^2 rotating pulse, 160 steps to t = 0.5, constant D, paper-literal aux term."""
    cfg = W.C1
    f = W.rotating_pulse(cfg)
    f["D"] = None
    g_gpu, g_orc, st = run_pair(cfg.N, cfg.N, f, cfg.steps, lbm.LBM_AUX_LOCAL)
    assert rel(g_gpu, g_orc) <= TOL64
    phi = O.phi(O.Problem(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D), g_orc)
    assert abs(st["mass"] - O.mass(phi)) <= 1e-13 * O.mass(phi)
    assert st["step"] == cfg.steps and st["nonfinite"] == 0


@pytest.mark.parametrize("aux", [lbm.LBM_AUX_LOCAL, lbm.LBM_AUX_FLUX, lbm.LBM_AUX_NONE])
@pytest.mark.parametrize("shape", [(70, 45), (130, 67), (64, 3)])
def test_fp64_ragged_variable_D(aux, shape):
    """Several 64-wide column tiles with a ragged tail, rows not a multiple of the walk, variable D,
    a non-uniform velocity field."""
    nx, ny = shape
    f = case_fields(nx, ny, seed=nx * 7 + ny)
    g_gpu, g_orc, _ = run_pair(nx, ny, f, 25, aux)
    assert rel(g_gpu, g_orc) <= TOL64


@pytest.mark.parametrize("shape", [(3, 3), (3, 5), (5, 3), (65, 4)])
def test_fp64_degenerate_sizes(shape):
    nx, ny = shape
    f = case_fields(nx, ny, seed=3, varD=False)
    for aux in (lbm.LBM_AUX_LOCAL, lbm.LBM_AUX_FLUX):
        g_gpu, g_orc, _ = run_pair(nx, ny, f, 10, aux)
        assert rel(g_gpu, g_orc) <= TOL64


def test_fp64_source_path_sec3_benchmark():
    """The Sec. 3 benchmark on its periodic proxy (N = 40, kappa = 0.05, Lambda = 1/12): time-dependent
    source S and dS/dt supplied per step."""
    N, kappa = 40, 0.05
    x1 = W.x1_problem(N, kappa)
    f = dict(dx=x1["dx"], dt=x1["dt"], ux=x1["ux"], uy=x1["uy"], phi0=x1["phi0"], D=None, D_const=kappa)
    g_gpu, g_orc, _ = run_pair(N, N, f, x1["steps"], lbm.LBM_AUX_LOCAL, lam=x1["lam"],
                               sources=lambda t: x1["source"](t * x1["dt"]))
    assert rel(g_gpu, g_orc) <= TOL64
    p = O.Problem(N, N, x1["dx"], x1["dt"], x1["lam"], kappa)
    er = O.rms_error(O.phi(p, g_gpu), x1["exact"](x1["steps"] * x1["dt"])) * N / (N + 1)
    assert abs(er / 3.679e-03 - 1) < 1e-3  # Table 2, Present, kappa = 0.05, N = 40


# ---- reduced precision against the FP64 oracle ----------------------------------------------------

@pytest.mark.parametrize("mode,bound", [("f64s_f32m", 2e-5), ("f32", 2e-5), ("f16s", 3e-3)])
def test_reduced_precision_vs_oracle(mode, bound):
    """64^2 pulse, 160 steps.  Bounds: FP32 math accumulates ~160 steps x a few ulp(2^-24) of the
    largest population; FP16 storage adds one rounding of 2^-11 relative per stored value per step,
    damped by the collision (measured values are reported by the benchmark)."""
    cfg = W.C1
    f = W.rotating_pulse(cfg)
    f["D"] = None
    g_gpu, g_orc, st = run_pair(cfg.N, cfg.N, f, cfg.steps, lbm.LBM_AUX_LOCAL, mode=mode)
    err = rel(g_gpu, g_orc)
    assert err <= bound, err
    assert st["nonfinite"] == 0


# ---- full-size one-step parity at the benchmark's launch configuration -----------------------------

def _one_step_after(nx, ny, f, mode, warm, aux=lbm.LBM_AUX_LOCAL):
    p = lbm.make_params(nx, ny, f["dx"], f["dt"], f["lam"], f["D_const"], mode, aux)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy")}
    if f.get("D") is not None:
        fields["D"] = dev(f["D"])
    s = Solver([(p, fields)])
    s.step(warm)
    g0 = s.populations()
    s.step(1)
    g1 = s.populations()
    s.close()
    return g0, g1


def _windows(n, size, seed):
    rng = np.random.default_rng(seed)
    starts = [(0, 0), (n - size // 2, n - size // 2)]  # one window across the periodic seam
    starts += [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(2)]
    return starts


def _gather(g, ys, xs):
    iy = torch.as_tensor(ys, device=g.device)
    ix = torch.as_tensor(xs, device=g.device)
    return g.index_select(1, iy).index_select(2, ix).cpu().numpy()


def _oracle_window_step(g0, f, y0, x0, w, m, lam, D_const, aux):
    """Oracle step on a (w + 2m)^2 window gathered with periodic wrap; only the inner w x w nodes
    (at distance >= m from the window edge) are valid."""
    n = g0.shape[-1]
    ys = (np.arange(y0 - m, y0 + w + m)) % n
    xs = (np.arange(x0 - m, x0 + w + m)) % n
    gw = _gather(g0, ys, xs)
    sub = lambda a: None if a is None else np.ascontiguousarray(a[np.ix_(ys, xs)])
    p = O.Problem(w + 2 * m, w + 2 * m, f["dx"], f["dt"], lam, D_const, aux)
    out = O.step(p, gw, sub(f["ux"]), sub(f["uy"]), sub(f.get("D")))
    # out holds g^{n+1}; nodes within m-1 of the edge see wrapped (wrong) neighbours
    return out[:, m:-m, m:-m], ys[m:-m], xs[m:-m]


@pytest.mark.parametrize("mode,tol,warm", [("f64", TOL64, 40), ("f32", 3e-6, 40), ("f32", 3e-6, 41)])
def test_full_size_2048_one_step(mode, tol, warm):
    """2048^2 pulse in the benchmark's launch configuration: after 40 (41) steps, one more GPU step
    equals one oracle step from the GPU state (every node is compared).  FP32 runs on one buffer in
    place, so the two warm-up counts cover both of its alternating steps and both state layouts."""
    cfg = W.C2
    f = W.rotating_pulse(cfg)
    f["D"] = None
    f["lam"] = cfg.lam
    g0, g1 = _one_step_after(cfg.N, cfg.N, f, mode, warm)
    p = O.Problem(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, O.AUX_LOCAL)
    want = O.step(p, g0.cpu().numpy(), f["ux"], f["uy"])
    assert rel(g1.cpu().numpy(), want) <= tol


@pytest.mark.parametrize("mode", ["f64", "f64s_f32m", "f32", "f16s"])
def test_full_size_8192_variable_D_windows(mode):
    """8192^2 with D(x) = 1e-3 (1 + 0.5 sin(pi x) sin(pi y)): one step after 10, checked on sampled
    64^2 windows (one across the periodic seam) against the oracle stepping the GPU state."""
    cfg = W.C3
    f = W.rotating_pulse(cfg)
    f["lam"] = cfg.lam
    g0, g1 = _one_step_after(cfg.N, cfg.N, f, mode, 10)
    gmax = float(g1.abs().max())  # normalisation: the largest population of the whole lattice
    for (y0, x0) in _windows(cfg.N, 64, seed=17):
        want, ys, xs = _oracle_window_step(g0, f, y0, x0, 64, 2, cfg.lam, cfg.D, O.AUX_LOCAL)
        got = _gather(g1, ys, xs)
        if mode == "f64":
            assert np.abs(got - want).max() <= TOL64 * gmax
        elif mode == "f16s":
            # one FP16 rounding (half an ulp: 2^-11 relative) of (g - w phi_ref) 2^15, plus the FP32
            # collision (a few 2^-24 of the largest value) and the FP16 subnormal spacing 2^-24 / 2^15
            bound = 2.0 ** -11 * np.abs(want) + 1e-6 * gmax + 2.0 ** -39
            assert np.all(np.abs(got - want) <= bound)
        else:
            assert np.abs(got - want).max() <= 1e-6 * gmax


@pytest.mark.parametrize("mode", ["f64", "f32", "f16s"])
def test_longest_row_windows(mode):
    """The longest row the ABI accepts (nx = 2^24, ny = 3): lane byte offsets and tile indices at their
    extremes (65,536 tiles per row, column bands of 8,192 tiles).  One step after 3, checked on
    windows at the start, the middle and the periodic end of the row against the oracle stepping the
    GPU state (all three rows, which wrap in y exactly as on the GPU); then two more steps in one fused
    launch (32,768 tiles of 512 columns), bitwise equal to two single steps."""
    nx, ny, w, m = 1 << 24, 3, 64, 2
    x = np.arange(nx) / nx
    ux = np.broadcast_to(0.2 * np.sin(2 * np.pi * x), (ny, nx)).copy()
    uy = np.broadcast_to(0.1 * np.cos(2 * np.pi * 3 * x), (ny, nx)).copy()
    uy[1] *= -1.0
    phi0 = 1.0 + 0.5 * np.broadcast_to(np.cos(2 * np.pi * 5 * x), (ny, nx))
    dx, dt, lam, D = 1.0 / nx, 0.5 / nx, 0.25, 1.0 / (6.0 * nx)
    p = lbm.make_params(nx, ny, dx, dt, lam, D, mode, phi_ref=1.0)
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(ux), "uy": dev(uy)})])
    assert s.get_launch()["fuse"] == 2  # one periodic instance: two steps per launch by default
    s.set_launch(1, 2, tile_width=256)  # one step per launch, column bands of 8,192 tiles
    s.step(3)
    g0 = s.populations()
    s.step(1)
    g1 = s.populations()
    img = s.state_save()
    s.step(2)  # two more single steps, then the same two steps in one fused launch (32,768 tiles per row)
    g3 = s.populations()
    s.state_load(img, 4)
    s.set_launch(4, 1, tile_width=512, fuse=2)
    s.step(2)
    assert torch.equal(s.populations(), g3)
    s.close()
    gmax = float(g1.abs().max())
    bound = {"f64": TOL64, "f32": 1e-6, "f16s": 2.0 ** -10}[mode]
    for x0 in (0, nx // 2 + 12345, nx - w // 2):
        xs = (np.arange(x0 - m, x0 + w + m)) % nx
        ix = torch.as_tensor(xs, device=g0.device)
        q = O.Problem(w + 2 * m, ny, dx, dt, lam, D, O.AUX_LOCAL)
        want = O.step(q, g0.index_select(2, ix).cpu().numpy(), ux[:, xs], uy[:, xs])[:, :, m:-m]
        got = g1.index_select(2, ix[m:-m]).cpu().numpy()
        err = np.abs(got - want).max() / gmax
        assert err <= bound, (x0, err)
    del g0, g1, g3
    torch.cuda.empty_cache()


def test_full_size_8192_flux_window():
    cfg = W.C3
    f = W.rotating_pulse(cfg)
    f["lam"] = cfg.lam
    g0, g1 = _one_step_after(cfg.N, cfg.N, f, "f64", 5, aux=lbm.LBM_AUX_FLUX)
    gmax = float(g1.abs().max())
    for (y0, x0) in _windows(cfg.N, 64, seed=19)[:2]:
        want, ys, xs = _oracle_window_step(g0, f, y0, x0, 64, 3, cfg.lam, cfg.D, O.AUX_FLUX)
        got = _gather(g1, ys, xs)
        assert np.abs(got - want).max() <= TOL64 * gmax


# ---- diagnostics ----------------------------------------------------------------------------------

def test_reduction_matches_fsum_and_oracle_definitions():
    cfg = W.PulseConfig(N=300, steps=30)
    f = W.rotating_pulse(cfg)
    p = lbm.make_params(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, "f64")
    s = Solver([(p, {k: dev(f[k]) for k in ("phi0", "ux", "uy")})])
    s.step(cfg.steps)
    ref = W.pulse_reference(cfg, f)
    st, phi = s.macros(ref=dev(ref), want_phi=True)
    s.close()
    phi = phi.cpu().numpy()
    m = O.mass(phi)
    assert abs(st["mass"] - m) <= 4 * math.ulp(m)
    for key, want in (("rms_err", O.rms_error(phi, ref)), ("l2_rel_err", O.l2_rel_error(phi, ref)),
                      ("max_abs_err", O.max_abs_error(phi, ref))):
        assert abs(st[key] - want) <= 4 * math.ulp(want), key
    assert st["max_abs_phi"] == np.abs(phi).max()


def test_reduction_compensation_on_cancelling_data():
    """phi0 mixing +-1e8 and +-1e-3 values (heavy cancellation): the compensated mass of the initial
    state equals the correctly rounded sum of the same phi values."""
    n = 256
    rng = np.random.default_rng(23)
    phi0 = rng.uniform(-1, 1, (n, n)) * np.where(rng.uniform(0, 1, (n, n)) < 0.5, 1e8, 1e-3)
    p = lbm.make_params(n, n, 1.0, 1.0, 0.25, 1e-9, "f64")
    z = np.zeros((n, n))
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(z), "uy": dev(z)})])
    st, phi = s.macros(want_phi=True)
    s.close()
    m = O.mass(phi.cpu().numpy())
    assert abs(st["mass"] - m) <= 4 * math.ulp(abs(m)) + 1e-300


# ---- FP16S codec against numpy's IEEE binary16 ------------------------------------------------------

def test_f16s_decode_exhaustive():
    """Every 16-bit code, loaded as raw state, decodes to h * 2^-k + w_i phi_ref computed in FP32."""
    n = 256  # 65536 nodes: every code once per plane
    k, phi_ref = 15, 0.75
    p = lbm.make_params(n, n, 1.0, 1.0, 0.25, 1e-3, "f16s", scale_log2=k, phi_ref=phi_ref)
    z = np.zeros((n, n))
    s = Solver([(p, {"phi0": dev(np.full((n, n), phi_ref)), "ux": dev(z), "uy": dev(z)})])
    codes = np.arange(65536, dtype=np.uint16).reshape(n, n)
    pitch = lbm.pitch_of(p)
    raw = np.zeros(lbm.lbm_state_bytes(s.ctx) // 2, np.uint16)
    img = raw[:n * 9 * pitch].reshape(n, 9, pitch)  # image layout [ny][9][pitch]
    for i in range(9):
        img[:, i, :n] = codes
    s.state_load(torch.from_numpy(raw.view(np.uint8)).cuda(), 0)
    g = s.populations().cpu().numpy()
    s.close()
    ex, ey, w = O.lattice()
    h = codes.view(np.float16).astype(np.float32)
    for i in range(9):
        want = (h * np.float32(2.0 ** -k) + np.float32(w[i] * phi_ref)).astype(np.float64)
        got = np.roll(g[i], (-int(ey[i]), -int(ex[i])), (0, 1))  # buf_i(y) = g_i(y + e_i)
        same = (got == want) | (np.isnan(got) & np.isnan(want))
        assert same.all(), i


@pytest.mark.parametrize("phi_ref", [0.0, 0.5])
def test_f16s_encode_matches_numpy_rne(phi_ref):
    """u = 0 makes the initial populations the FP32 products w_i phi0; the encoder subtracts the
    FP32 shift w_i phi_ref (a separate rounding, never fused with the product), scales by 2^k (exact)
    and rounds to FP16.  The stored codes equal numpy's round-to-nearest-even float16 of the same FP32
    value, formed here with numpy's IEEE float32 arithmetic."""
    n = 1024
    k = 15
    rng = np.random.default_rng(29)
    phi0 = rng.uniform(-1.0, 3.0, (n, n))
    z = np.zeros((n, n))
    p = lbm.make_params(n, n, 1.0, 1.0, 0.25, 1e-3, "f16s", scale_log2=k, phi_ref=phi_ref)
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(z), "uy": dev(z)})])
    raw = s.state_save().cpu().numpy().view(np.uint16)
    s.close()
    pitch = lbm.pitch_of(p)
    img = raw[:n * 9 * pitch].reshape(n, 9, pitch)
    ex, ey, w = O.lattice()
    p32 = phi0.astype(np.float32)
    for i in range(9):
        d32 = np.float32(w[i]) * p32 - np.float32(w[i] * phi_ref)  # two FP32 roundings
        want = (d32 * np.float32(2.0 ** k)).astype(np.float16).view(np.uint16)
        got = np.roll(img[:, i, :n], (int(ey[i]), int(ex[i])), (0, 1))
        assert np.array_equal(got, want), i


# ---- failure handling, checkpoints, determinism ----------------------------------------------------

def test_nonfinite_phi_is_reported():
    n = 32
    phi0 = np.ones((n, n))
    phi0[5, 7] = np.nan
    z = np.zeros((n, n))
    p = lbm.make_params(n, n, 1.0, 1.0, 0.25, 1e-3, "f64")
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(z), "uy": dev(z)})])
    s.step(3)
    with pytest.raises(lbm.LbmError) as ei:
        s.macros()
    assert ei.value.status == lbm.LBM_E_NONFINITE
    st = s.macros(raise_nonfinite=False)
    assert st["nonfinite"] > 0 and st["status"] == lbm.LBM_E_NONFINITE
    s.close()


def test_invalid_fields_rejected_at_init():
    n = 16
    z = np.zeros((n, n))
    D = np.full((n, n), 1e-3)
    D[3, 3] = -1e-3
    p = lbm.make_params(n, n, 1.0, 1.0, 0.25, 1e-3, "f64")
    with pytest.raises(lbm.LbmError, match="D field"):
        Solver([(p, {"phi0": dev(np.ones((n, n))), "ux": dev(z), "uy": dev(z), "D": dev(D)})])
    p = lbm.make_params(n, n, 1.0, 1.0, 0.25, 1e-3, "f16s", scale_log2=24)
    with pytest.raises(lbm.LbmError, match="does not fit FP16"):
        Solver([(p, {"phi0": dev(np.ones((n, n))), "ux": dev(z), "uy": dev(z)})])


@pytest.mark.parametrize("mode", ["f64", "f16s"])
def test_checkpoint_resume_and_determinism(mode):
    cfg = W.PulseConfig(N=96, steps=30, D_variable=True)
    f = W.rotating_pulse(cfg)
    p = lbm.make_params(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, mode)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy", "D")}
    a = Solver([(p, fields)])
    a.step(10)
    ck = a.state_save()
    a.step(20)
    end_a = a.state_save()
    b = Solver([(p, fields)])
    b.state_load(ck, 10)
    b.step(20)
    end_b = b.state_save()
    assert b.macros()["step"] == 30
    assert torch.equal(end_a, end_b)
    c = Solver([(p, fields)])
    c.step(30)
    assert torch.equal(c.state_save(), end_a)
    for s in (a, b, c):
        s.close()


def test_multi_instance_context_matches_single():
    cfgs = [W.PulseConfig(N=48, steps=12), W.PulseConfig(N=80, steps=12, U0=2.0, D=3e-3)]
    inst = []
    for cfg in cfgs:
        f = W.rotating_pulse(cfg)
        inst.append((lbm.make_params(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, "f64"),
                     {k: dev(f[k]) for k in ("phi0", "ux", "uy")}))
    both = Solver(inst)
    both.step(12)
    for k, one in enumerate(inst):
        s = Solver([one])
        s.step(12)
        assert torch.equal(s.populations(), both.populations(k))
        s.close()
    both.close()


def test_graph_replay_matches_eager_steps():
    """lbm_step replays a captured graph for long runs; interleaved with eager work and syncs, every
    replay leaves exactly the state that single eager steps produce."""
    cfg = W.PulseConfig(N=96, steps=0, D_variable=True)
    f = W.rotating_pulse(cfg)
    p = lbm.make_params(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, "f32")
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy", "D")}
    a = Solver([(p, fields)])
    b = Solver([(p, fields)])
    for rep, n in enumerate((64, 65, 96, 64)):
        a.step(n)                      # graph replays (+ eager remainder)
        for _ in range(n):
            b.step(1)                  # eager only
        a.macros()                     # synchronizing work between replays
        assert torch.equal(a.state_save(), b.state_save()), rep
    a.close()
    b.close()


def test_launch_defaults_and_bad_launch_shapes():
    cfg = W.PulseConfig(N=64, steps=0)
    f = W.rotating_pulse(cfg)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy")}
    def launch(rows, remap, width, cap, h=0, stores=1, fuse=1):
        return {"rows": rows, "xcd_remap": remap, "tile_width": width, "max_waves": cap, "xcd_rows": h,
                "stores": stores, "fuse": fuse}

    def fused(nx, ny, stores, mode):  # two steps per launch: the tile shapes of the sweeps
        narrow = (nx + 255) // 256 <= 8
        width, rows = {"f32": (512, 16), "f16s": (512, 16) if narrow else (256, 24),
                       "f16sr": (512, 16) if narrow else (256, 24),
                       "f64s_f32m": (512, 32) if narrow else (512, 16)}.get(mode, (256, 32) if narrow else (512, 16))
        while width > 128 and width // 2 >= nx:
            width //= 2
        want = 256 if mode in ("f64", "f64s_f32m") and width == 512 else 512  # two tiles per CU
        while rows > 4 and -(-nx // width) * -(-ny // rows) < want:
            rows //= 2
        while width > 128 and -(-nx // width) * -(-ny // rows) < 256:
            width //= 2
        return launch(rows, 1, width, 0, 0, stores, 2)

    # One periodic D2Q9 TRT-R instance of at least 2^18 nodes (2^21 with FP16 storage) runs two steps per
    # launch; a smaller one runs one.  A context that touches at most 256 MiB per step is served by the
    # Infinity Cache: cached stores, row bands, every wave resident (64-column tiles kept for FP64
    # storage on narrow lattices).
    for mode, w in (("f32", launch(1, 1, 256, 0)), ("f64", launch(1, 1, 64, 0)), ("f16s", launch(1, 1, 256, 0))):
        s = Solver([(lbm.make_params(64, 64, f["dx"], f["dt"], cfg.lam, cfg.D, mode), fields)])
        assert s.get_launch() == w, mode
        s.close()
    for n, mode, w in ((725, "f32", None), (725, "f64", None), (725, "f16s", launch(1, 1, 256, 0)),
                       (512, "f32", None), (512, "f64", None), (511, "f64", launch(1, 1, 64, 0)),
                       (1449, "f16s", None), (1448, "f16s", launch(1, 1, 256, 0))):
        big = {k: dev(np.resize(v.cpu().numpy(), (n, n))) for k, v in fields.items()}
        s = Solver([(lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode), big)])
        l2 = mode == "f32" and n * n * 80 <= 32 << 20  # FP32 within the L2 caches streams its stores
        assert s.get_launch() == (w or fused(n, n, 0 if l2 else 1, mode)), (n, mode)
        s.close()
        del big
    for mode, w in (("f32", launch(1, 1, 256, 0)), ("f64", launch(1, 1, 64, 0)), ("f16s", launch(1, 1, 256, 0))):
        s = Solver([(lbm.make_params(64, 64, f["dx"], f["dt"], cfg.lam, cfg.D, mode, boundary=lbm.LBM_BC_NEE), fields)])
        assert s.get_launch() == w, mode
        s.close()
    s = Solver([(lbm.make_params(64, 64, f["dx"], f["dt"], cfg.lam, cfg.D, "f32", lbm.LBM_AUX_FLUX), fields)])
    assert s.get_launch() == launch(2, 1, 256, 0)  # the flux form in one step per launch (a small lattice)
    s.close()
    s = Solver([(lbm.make_params(64, 64, f["dx"], f["dt"], cfg.lam, cfg.D, "f32", tau3=0.7), fields)])
    assert s.get_launch() == launch(1, 1, 256, 0)  # MRT-R: one step per launch
    s.close()

    # Larger contexts stream (non-temporal stores).  One-step launches with 4 or more wide tiles per row:
    # row blocks (FP32 about 64 tiles each, FP64 about 32; FP16 keeps column bands at 8 and 16 tiles per
    # row); FP32 with a D(x) field runs 6 waves per SIMD.  Narrower FP64: 64-column tiles in hardware
    # order.  (Sizes: more than 256 MiB even with one population buffer; boundary instances never run in
    # place.)
    def fields_of(nx, ny, var=False):
        src = dict(f, D=np.full_like(f["phi0"], cfg.D))
        keys = ("phi0", "ux", "uy", "D") if var else ("phi0", "ux", "uy")
        return {k: dev(np.ascontiguousarray(np.resize(src[k], (ny, nx)))) for k in keys}

    for nx, ny, mode, var, bc, tau3, w in (
            (2048, 1700, "f32", False, 0, 0.0, fused(2048, 1700, 0, "f32")),
            (2048, 1700, "f32", False, 0, 0.8, launch(1, 1, 256, 0, 0, 2)),  # MRT-R: one buffer in place
            (2048, 3000, "f32", False, 0, 0.8, launch(1, 3, 256, 5, 8, 0)),
            (2048, 1500, "f64", False, 0, 0.0, fused(2048, 1500, 0, "f64")),
            (2048, 1500, "f64", False, 0, 0.8, launch(1, 3, 256, 4, 4, 0)),
            (1024, 3000, "f64", False, 0, 0.8, launch(1, 3, 256, 4, 8, 0)),
            (768, 4000, "f64", False, 0, 0.8, launch(1, 0, 64, 4, 0, 0)),
            (2048, 5100, "f16s", False, 0, 0.8, launch(1, 2, 256, 0, 0, 0)),
            (2049, 3000, "f32", False, 0, 0.8, launch(1, 3, 256, 5, 7, 0)),
            (2049, 5100, "f16s", False, 0, 0.0, fused(2049, 5100, 0, "f16s")),
            (2049, 5100, "f16s", False, 0, 0.8, launch(1, 3, 256, 0, 3, 0)),
            (8192, 800, "f32", False, 0, 0.8, launch(1, 3, 256, 5, 2, 0)),
            (4096, 1500, "f32", True, 0, 0.8, launch(1, 3, 256, 6, 4, 0)),
            (2048, 1700, "f32", False, lbm.LBM_BC_NEE, 0.0, launch(1, 3, 256, 5, 4, 0)),
            (2048, 900, "f64", False, lbm.LBM_BC_NEE, 0.0, launch(1, 3, 256, 0, 2, 0))):
        fl = fields_of(nx, ny, var)
        s = Solver([(lbm.make_params(nx, ny, f["dx"], f["dt"], cfg.lam, cfg.D, mode, boundary=bc, tau3=tau3), fl)])
        assert s.get_launch() == w, (nx, ny, mode, var, bc, tau3)
        s.close()
        del fl
    two = [(lbm.make_params(64, 64, f["dx"], f["dt"], cfg.lam, cfg.D, "f32"), fields)] * 2
    s = Solver(two)  # a uniform batch: two steps per launch in 128 x 16 tiles
    assert s.get_launch(1) == launch(16, 1, 128, 0, 0, 1, 2)
    with pytest.raises(lbm.LbmError) as ei:  # a batch fuses as a whole or not at all
        s.set_launch(16, 1, inst=0, tile_width=128, fuse=2)
    assert ei.value.status == lbm.LBM_E_ARG
    s.set_launch(1, 1, tile_width=64)  # one step per launch: the batched kernel's 64-column tiles
    assert s.get_launch(1) == launch(1, 1, 64, 0, 0, 0)
    s.set_launch(1, 3, tile_width=256, xcd_rows=4)
    assert s.get_launch(0) == launch(1, 3, 256, 0, 4, stores=0)
    s.set_launch(1, 2, tile_width=256, xcd_rows=4, stores=1)  # xcd_rows only counts with order 3
    assert s.get_launch(1) == launch(1, 2, 256, 0)
    for remap, kw in ((1, dict(tile_width=128)), (1, dict(tile_width=0)), (1, dict(max_waves=2)),
                      (1, dict(max_waves=9)), (1, dict(max_waves=-1)), (3, {}), (3, dict(xcd_rows=65)),
                      (3, dict(xcd_rows=-2)), (4, {}), (-1, {}), (1, dict(stores=2)), (1, dict(stores=-1)),
                      (1, dict(fuse=2, tile_width=64))):
        with pytest.raises(lbm.LbmError) as ei:
            s.set_launch(1, remap, **kw)
        assert ei.value.status == lbm.LBM_E_ARG, (remap, kw)
    s.close()


@pytest.mark.parametrize("mode", ["f32", "f16s", "f64"])
def test_xcd_tile_orders_do_not_change_results(mode):
    """The four block-to-tile orders (hardware, row bands, column bands, row blocks) on a lattice whose
    tile rows hold 8 tiles (256-column tiles) or 32 (64-column tiles), so that column bands apply, with
    ragged last tiles in x and y and row blocks that leave a remainder in hardware order: bitwise
    equal states."""
    nx, ny = 2000, 37
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    p = lbm.make_params(nx, ny, dx, dx / 10, 0.25, 1e-3, mode)
    fields = {"phi0": dev(np.exp(-((X - 0.3) ** 2 + Y ** 2) / 0.02)), "ux": dev(-np.pi * Y), "uy": dev(np.pi * X)}
    states = []
    for remap, width, rows, h, stores in ((0, 256, 1, 0, 0), (1, 256, 1, 0, 1), (2, 256, 1, 0, 0), (2, 64, 1, 0, 1),
                                          (2, 64, 3, 0, 0), (2, 256, 2, 0, 1), (3, 256, 1, 2, 0), (3, 256, 1, 1, 1),
                                          (3, 64, 1, 1, 0), (3, 256, 2, 1, 1), (3, 256, 1, 64, 0)):
        s = Solver([(p, fields)])
        s.set_launch(rows, remap, tile_width=width, xcd_rows=h, stores=stores)
        s.step(25)
        states.append(s.state_save())
        s.close()
    for st in states[1:]:
        assert torch.equal(st, states[0])


@pytest.mark.parametrize("mode,aux", [("f64", lbm.LBM_AUX_LOCAL), ("f16s", lbm.LBM_AUX_LOCAL),
                                      ("f64", lbm.LBM_AUX_FLUX), ("f32", lbm.LBM_AUX_FLUX)])
def test_launch_shape_does_not_change_results(mode, aux):
    cfg = W.PulseConfig(N=200, steps=0, D_variable=True)
    f = W.rotating_pulse(cfg)
    p = lbm.make_params(cfg.N, cfg.N - 37, f["dx"], f["dt"], cfg.lam, cfg.D, mode, aux)
    fields = {k: dev(np.ascontiguousarray(f[k][:cfg.N - 37])) for k in ("phi0", "ux", "uy", "D")}
    states = []
    for rows, remap, width, cap, h, st in ((1, 0, 64, 0, 0, 0), (4, 1, 64, 6, 0, 1), (7, 1, 256, 0, 0, 0),
                                           (64, 0, 64, 0, 0, 1), (1, 1, 256, 5, 0, 0), (3, 0, 256, 8, 0, 0),
                                           (1, 3, 256, 5, 2, 1), (2, 3, 64, 4, 3, 0)):
        s = Solver([(p, fields)])
        s.set_launch(rows, remap, tile_width=width, max_waves=cap, xcd_rows=h, stores=st)
        assert s.get_launch() == {"rows": rows, "xcd_remap": remap, "tile_width": width, "max_waves": cap,
                                  "xcd_rows": h, "stores": st, "fuse": 1}
        s.step(70)
        states.append(s.state_save())
        s.close()
    for st in states[1:]:
        assert torch.equal(st, states[0])


def test_bench_copy_is_a_copy():
    a = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    lbm.lbm_bench_copy(b, a)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
