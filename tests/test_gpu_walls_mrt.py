"""Walls by halfway anti-bounce-back and the MRT-R operator on the HIP path, through the C ABI,
against the FP64 oracle on the same seeded inputs; the slip-free free parameter of Sec. 3.3 on the
GPU."""
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


def wall_case(nx, ny, seed):
    """A pulse in a shear flow between walls (x periodic) with variable D, per-column wall values
    that move in time (equal to phi0's rows at t = 0) and a time-dependent source."""
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    rng = np.random.default_rng(seed)
    c = 4.0
    ux = c * (0.25 - 0.3 * Y + 0.1 * np.sin(np.pi * X))
    uy = c * (0.15 * np.cos(np.pi * X))
    phi0 = 0.3 + np.exp(-((X - 0.2) ** 2 + (Y + 0.1) ** 2) / 0.1)
    D = 2e-3 * (1 + 0.5 * rng.uniform(-1, 1, (ny, nx)))
    S0 = rng.uniform(-1, 1, (ny, nx))

    def phi_w(t):
        return phi0 * (1.0 + 0.3 * t) + 0.05 * np.sin(3.0 * X) * t

    def source(t):
        return S0 * np.cos(4.0 * t), -4.0 * S0 * np.sin(4.0 * t)

    return dict(dx=dx, dt=dx / c, ux=ux, uy=uy, phi0=phi0, D=D, D_const=2e-3, phi_w=phi_w, source=source)


def run_wall_pair(nx, ny, f, steps, mode="f64", aux=lbm.LBM_AUX_LOCAL, tau3=0.0, rows=None, lam=0.25):
    """GPU: the wall values of the current state are set before each step (t_0's are phi0's, the
    default).  Oracle: each step writes the reflected populations of the new state with the wall
    values of the new time level."""
    p = lbm.make_params(nx, ny, f["dx"], f["dt"], lam, f["D_const"], mode, aux, boundary=lbm.LBM_BC_WALLS, tau3=tau3)
    s = Solver([(p, {k: dev(f[k]) for k in ("phi0", "ux", "uy", "D")})])
    if rows is not None:  # rows per wave, or (rows, xcd_remap, tile_width, xcd_rows, stores)
        r, remap, width, h, st = rows if isinstance(rows, tuple) else (rows, 1, 64, 0, 0)
        s.set_launch(r, remap, tile_width=width, xcd_rows=h, stores=st)
    op = O.Problem(nx, ny, f["dx"], f["dt"], lam, f["D_const"], aux, O.BC_WALLS, tau3)
    g = O.init(op, f["phi0"], f["ux"], f["uy"])
    for n in range(steps):
        t = n * f["dt"]
        S, dS = f["source"](t)
        if n > 0:
            s.set_dirichlet(dev(f["phi_w"](t)))
        s.step(1, S=[dev(S)], dSdt=[dev(dS)])
        g = O.step(op, g, f["ux"], f["uy"], f["D"], S, dS, phi_b=f["phi_w"](t + f["dt"]))
    s.set_dirichlet(dev(f["phi_w"](steps * f["dt"])))
    g_gpu = s.populations().cpu().numpy()
    st = s.macros()
    s.close()
    return g_gpu, g, st


@pytest.mark.parametrize("shape", [(70, 45), (130, 67), (3, 3), (64, 5)])
def test_walls_fp64_parity(shape):
    nx, ny = shape
    f = wall_case(nx, ny, 21 + nx)
    g_gpu, g_orc, _ = run_wall_pair(nx, ny, f, 25)
    assert rel(g_gpu, g_orc) <= TOL64


def test_walls_initial_state_is_the_equilibrium():
    f = wall_case(70, 45, 3)
    p = lbm.make_params(70, 45, f["dx"], f["dt"], 0.25, f["D_const"], "f64", boundary=lbm.LBM_BC_WALLS)
    s = Solver([(p, {k: dev(f[k]) for k in ("phi0", "ux", "uy")})])
    g = s.populations().cpu().numpy()
    s.close()
    op = O.Problem(70, 45, f["dx"], f["dt"], 0.25, f["D_const"], O.AUX_LOCAL, O.BC_WALLS)
    assert rel(g, O.init(op, f["phi0"], f["ux"], f["uy"])) <= 1e-15


@pytest.mark.parametrize("rows", [2, 4, (1, 3, 256, 1, 1), (1, 3, 64, 2, 0)])
def test_walls_launch_shape_does_not_change_results(rows):
    f = wall_case(97, 70, 4)
    a, _, _ = run_wall_pair(97, 70, f, 10, rows=1)
    b, _, _ = run_wall_pair(97, 70, f, 10, rows=rows)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("mode,bound", [("f32", 2e-5), ("f16s", 1e-2)])
def test_walls_reduced_precision(mode, bound):
    f = wall_case(70, 45, 8)
    g_gpu, g_orc, _ = run_wall_pair(70, 45, f, 40, mode=mode)
    err = rel(g_gpu, g_orc)
    print(f"walls {mode}: normalised max error vs FP64 oracle {err:.3e}")
    assert err <= bound


def _channel(tau1, tau2, mode="f64", nx=64, ny=24, phi_bot=0.3, phi_top=0.7, S0=2e-3, max_steps=400000):
    """Steady diffusion across a channel between walls at y = -1/2 and y = ny - 1/2 (lattice units,
    dx = dt = 1), uniform source, u = 0; returns the relative RMS error against the exact
    linear-plus-parabolic profile and the number of steps to convergence."""
    kappa = (tau1 - 0.5) / 3.0
    p = lbm.make_params(nx, ny, 1.0, 1.0, (tau1 - 0.5) * (tau2 - 0.5), kappa, mode, lbm.LBM_AUX_LOCAL,
                        boundary=lbm.LBM_BC_WALLS)
    z = np.zeros((ny, nx))
    s = Solver([(p, {"phi0": dev(np.full((ny, nx), 0.5)), "ux": dev(z), "uy": dev(z)})])
    pb = np.full((ny, nx), 0.5)
    pb[0, :], pb[-1, :] = phi_bot, phi_top
    s.set_dirichlet(dev(pb))
    S = dev(np.full((ny, nx), S0))
    prev, steps = None, 0
    tol = 1e-15 if mode == "f64" else 1e-6
    while steps < max_steps:
        s.step(4096, S=[S])
        steps += 4096
        _, phi = s.macros(want_phi=True)
        phi = phi.cpu().numpy()
        if prev is not None and np.abs(phi - prev).max() < tol:
            break
        prev = phi
    s.close()
    y = np.arange(ny)[:, None] + 0.5
    exact = phi_bot + (phi_top - phi_bot) * y / ny + S0 / (2 * kappa) * y * (ny - y)
    return float(np.sqrt(np.mean((phi - exact) ** 2)) / np.abs(exact).max()), steps


def test_slip_free_parameter_on_the_gpu():
    """Sec. 3.3: with tau1 = 0.8 the free relaxation time tau2 = 1.375 makes the halfway
    anti-bounce-back walls slip-free (round-off error), and tau2 off it does not.  In FP32 the
    converged profile carries the storage rounding of the ~1e-1 populations, amplified by the
    ~ny^2/kappa steps of diffusion that set it (measured 3.3e-5), still well below the FP64 wall
    error off the slip-free value."""
    err, steps = _channel(0.8, 1.375)
    print(f"tau2 = 1.375: relative RMS error {err:.3e} after {steps} steps")
    assert err < 1e-11
    off = []
    for tau2 in (1.2, 1.55):
        e, _ = _channel(0.8, tau2)
        print(f"tau2 = {tau2}: relative RMS error {e:.3e}")
        assert e > 1e-4
        off.append(e)
    e32, _ = _channel(0.8, 1.375, "f32")
    print(f"FP32, tau2 = 1.375: relative RMS error {e32:.3e}")
    assert e32 < 1e-4 and e32 < 0.2 * min(off)


def mrt_pair(nx, ny, aux, tau3, steps=20, boundary=lbm.LBM_BC_PERIODIC):
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    rng = np.random.default_rng(nx + 100 * aux)
    c = 4.0
    ux, uy = c * 0.3 * np.sin(np.pi * Y), c * 0.2 * np.cos(np.pi * X)
    phi0 = 0.3 + np.exp(-((X - 0.1) ** 2 + Y ** 2) / 0.05)
    D = 3e-3 * (1 + 0.5 * rng.uniform(-1, 1, (ny, nx)))
    p = lbm.make_params(nx, ny, dx, dx / c, 0.2, 3e-3, "f64", aux, boundary=boundary, tau3=tau3)
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(ux), "uy": dev(uy), "D": dev(D)})])
    s.step(steps)
    g_gpu = s.populations().cpu().numpy()
    s.close()
    op = O.Problem(nx, ny, dx, dx / c, 0.2, 3e-3, aux, boundary, tau3)
    pb = phi0 if boundary == lbm.LBM_BC_WALLS else None
    g = O.run(op, O.init(op, phi0, ux, uy), steps, ux, uy, D, phi_b=pb)
    return g_gpu, g


@pytest.mark.parametrize("aux", [lbm.LBM_AUX_LOCAL, lbm.LBM_AUX_FLUX, lbm.LBM_AUX_NONE])
@pytest.mark.parametrize("tau3", [0.7, 1.6])
def test_mrt_fp64_parity(aux, tau3):
    g_gpu, g_orc = mrt_pair(70, 45, aux, tau3)
    assert rel(g_gpu, g_orc) <= TOL64


def test_mrt_with_walls_parity():
    g_gpu, g_orc = mrt_pair(66, 40, lbm.LBM_AUX_LOCAL, 0.9, boundary=lbm.LBM_BC_WALLS)
    assert rel(g_gpu, g_orc) <= TOL64


def test_tau3_one_is_trt_r():
    a, _ = mrt_pair(70, 45, lbm.LBM_AUX_LOCAL, 1.0)
    b, _ = mrt_pair(70, 45, lbm.LBM_AUX_LOCAL, 0.0)
    assert np.array_equal(a, b)


def test_walls_mrt_and_periodic_instances_share_a_context():
    f = wall_case(70, 45, 9)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy", "D")}
    ps = [lbm.make_params(70, 45, f["dx"], f["dt"], 0.25, f["D_const"], "f64", boundary=lbm.LBM_BC_WALLS),
          lbm.make_params(70, 45, f["dx"], f["dt"], 0.25, f["D_const"], "f64", tau3=0.8),
          lbm.make_params(70, 45, f["dx"], f["dt"], 0.25, f["D_const"], "f64")]
    both = Solver([(p, fields) for p in ps])
    both.step(9)
    got = [both.populations(i).cpu().numpy() for i in range(3)]
    both.close()
    for k, p in enumerate(ps):
        s = Solver([(p, fields)])
        s.step(9)
        assert np.array_equal(s.populations().cpu().numpy(), got[k])
        s.close()


def test_walls_and_mrt_errors():
    f = wall_case(16, 16, 1)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy")}
    mk = lambda **kw: lbm.make_params(16, 16, f["dx"], f["dt"], 0.25, 1e-3, "f64", **kw)
    with pytest.raises(lbm.LbmError) as ei:
        Solver([(mk(aux=lbm.LBM_AUX_FLUX, boundary=lbm.LBM_BC_WALLS), fields)])
    assert ei.value.status == lbm.LBM_E_UNSUPPORTED
    for bad in (0.4, float("nan"), -1.0):
        with pytest.raises(lbm.LbmError) as ei:
            Solver([(mk(tau3=bad), fields)])
        assert ei.value.status == lbm.LBM_E_ARG
    for kw in (dict(tau3=0.7), dict(boundary=lbm.LBM_BC_WALLS)):
        s = Solver([(mk(**kw), fields)])
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_adjoint_bytes(s.ctx)
        assert ei.value.status == lbm.LBM_E_UNSUPPORTED
        s.close()
