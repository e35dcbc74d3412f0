"""The D3Q19 and D3Q27 steps on the HIP path, through the C ABI, against the three-dimensional FP64
oracle on the same seeded inputs: FP64 parity (1e-12, normalised max-abs over all 19 or 27 planes)
on ragged and degenerate lattices with variable D, sources and both aux forms; FP32 bounds;
full-size windows at 256^3; graph replay, checkpoints, mixed contexts and error paths."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2312_10316_amd import Solver, lbm

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
LATTICES = [19, 27]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def case3(nx, ny, nz, seed, varD=True):
    """Seeded smooth fields on [-1, 1)^3: a rotation about an oblique axis plus a shear, a pulse on a
    background, and a variable D."""
    X, Y, Z, dx = W.mesh3(nx, ny, nz, -1.0, 1.0)
    rng = np.random.default_rng(seed)
    c = 4.0
    w = rng.uniform(-1, 1, 3)
    w = 0.6 * w / np.linalg.norm(w)
    u = c * 0.25 * np.stack([w[1] * Z - w[2] * Y + 0.1 * np.sin(np.pi * Y),
                            w[2] * X - w[0] * Z,
                            w[0] * Y - w[1] * X + 0.1 * np.cos(np.pi * X)])
    phi0 = 0.3 + np.exp(-((X - 0.2) ** 2 + (Y + 0.1) ** 2 + (Z - 0.3) ** 2) / 0.15)
    D = 2e-3 * (1 + 0.5 * rng.uniform(-1, 1, X.shape)) if varD else None
    return dict(dx=dx, dt=dx / c, u=u, phi0=phi0, D=D, D_const=2e-3, shape=X.shape)


def solver3(f, mode="f64", aux=lbm.LBM_AUX_LOCAL, lam=0.25, q=19):
    nz, ny, nx = f["shape"]
    p = lbm.make_params(nx, ny, f["dx"], f["dt"], lam, f["D_const"], mode, aux, nz=nz, lattice=q)
    fields = {"phi0": dev(f["phi0"]), "ux": dev(f["u"][0]), "uy": dev(f["u"][1]), "uz": dev(f["u"][2])}
    if f["D"] is not None:
        fields["D"] = dev(f["D"])
    return Solver([(p, fields)]), p


def oracle3(f, aux=lbm.LBM_AUX_LOCAL, lam=0.25, q=19):
    nz, ny, nx = f["shape"]
    return O.Problem3(nx, ny, nz, f["dx"], f["dt"], lam, f["D_const"], aux, q)


def run_pair3(f, steps, mode="f64", aux=lbm.LBM_AUX_LOCAL, source=None, q=19):
    s, _ = solver3(f, mode, aux, q=q)
    op = oracle3(f, aux, q=q)
    g = O.init3(op, f["phi0"], f["u"])
    if source is None:
        s.step(steps)
        g = O.run3(op, g, steps, f["u"], f["D"])
    else:
        for n in range(steps):
            S, dS = source(n)
            s.step(1, S=[dev(S)], dSdt=[dev(dS)])
            g = O.step3(op, g, f["u"], f["D"], S, dS)
    g_gpu = s.populations().cpu().numpy()
    st, phi = s.macros(want_phi=True)
    s.close()
    return g_gpu, g, st, phi.cpu().numpy(), op


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("aux", [lbm.LBM_AUX_LOCAL, lbm.LBM_AUX_NONE])
@pytest.mark.parametrize("shape", [(70, 6, 5), (130, 3, 4), (64, 4, 3), (3, 3, 3)])
def test_3d_fp64_parity(shape, aux, q):
    nx, ny, nz = shape
    f = case3(nx, ny, nz, 5 + nx + ny)
    g_gpu, g_orc, st, phi, op = run_pair3(f, 12, aux=aux, q=q)
    assert g_gpu.shape == (q, nz, ny, nx)
    assert rel(g_gpu, g_orc) <= TOL64
    phi_orc = O.phi3(op, g_orc)
    assert abs(st["mass"] - math.fsum(phi_orc.ravel())) <= 1e-12 * abs(st["mass"])
    assert np.abs(phi - phi_orc).max() <= 1e-12 * np.abs(phi_orc).max()


@pytest.mark.parametrize("q", LATTICES)
def test_3d_source_path(q):
    f = case3(66, 5, 4, 17)
    rng = np.random.default_rng(3)
    S0 = rng.uniform(-1, 1, f["shape"])
    src = lambda n: (S0 * math.cos(0.3 * n), -0.3 * S0 * math.sin(0.3 * n) / f["dt"])
    g_gpu, g_orc, _, _, _ = run_pair3(f, 10, source=src, q=q)
    assert rel(g_gpu, g_orc) <= TOL64


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("mode,bound", [("f64s_f32m", 2e-5), ("f32", 2e-5), ("f16s", 3e-3)])
def test_3d_reduced_precision(mode, bound, q):
    f = case3(70, 6, 5, 23)
    g_gpu, g_orc, _, _, _ = run_pair3(f, 40, mode=mode, q=q)
    err = rel(g_gpu, g_orc)
    print(f"D3Q{q} {mode}: normalised max error vs FP64 oracle {err:.3e}")
    assert err <= bound


@pytest.mark.parametrize("q", LATTICES)
def test_3d_set_velocity(q):
    f = case3(40, 5, 4, 31)
    s, _ = solver3(f, q=q)
    op = oracle3(f, q=q)
    g = O.init3(op, f["phi0"], f["u"])
    s.step(5)
    g = O.run3(op, g, 5, f["u"], f["D"])
    u2 = np.stack([f["u"][1], -f["u"][0], 0.5 * f["u"][2]])
    s.set_velocity(dev(u2[0]), dev(u2[1]), dev(u2[2]))
    s.step(5)
    g = O.run3(op, g, 5, u2, f["D"])
    got = s.populations().cpu().numpy()
    s.close()
    assert rel(got, g) <= TOL64


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("mode", ["f64", "f32", "f16s"])
def test_3d_full_size_256_windows(mode, q):
    """The 256^3 rotating pulse at its benchmark launch configuration: after 40 steps, one more step
    is compared on 10^3 windows (one across the periodic corner) with the oracle run on the 14^3
    block around each window, taken from the GPU state (two halo layers: the oracle wraps within
    the block, which spoils the velocity differences of its outermost layer, whose post-collision
    values reach the next layer)."""
    cfg = W.C6
    f3 = W.rotating_pulse3(cfg)
    n = cfg.N
    p = lbm.make_params(n, n, f3["dx"], f3["dt"], cfg.lam, cfg.D, mode, nz=n, lattice=q)
    u = f3["u"]
    s = Solver([(p, {"phi0": dev(f3["phi0"]), "ux": dev(u[0]), "uy": dev(u[1]), "uz": dev(u[2])})])
    s.step(40)
    g0 = s.populations()
    s.step(1)
    g1 = s.populations()
    s.close()
    gmax = float(g1.abs().max())
    w = 10
    for (z0, y0, x0) in [(128, 100, 150), (0, 0, 0), (250, 37, 255), (60, 200, 13)]:
        iz = [(z0 - 2 + k) % n for k in range(w + 4)]
        iy = [(y0 - 2 + k) % n for k in range(w + 4)]
        ix = [(x0 - 2 + k) % n for k in range(w + 4)]
        idx = np.ix_(iz, iy, ix)
        blk = g0[:, torch.tensor(iz)][:, :, torch.tensor(iy)][:, :, :, torch.tensor(ix)].cpu().numpy()
        want_full = g1[:, torch.tensor(iz)][:, :, torch.tensor(iy)][:, :, :, torch.tensor(ix)].cpu().numpy()
        op = O.Problem3(w + 4, w + 4, w + 4, f3["dx"], f3["dt"], cfg.lam, cfg.D, O.AUX_LOCAL, q)
        ub = np.stack([c[idx] for c in u])
        got = O.step3(op, blk, ub)
        inner = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
        if mode == "f16s":
            # one FP16 rounding (2^-11 relative) of g 2^15 after the FP32 collision, and the subnormal spacing
            bound = 2.0 ** -11 * np.abs(got[inner]) + 1e-6 * gmax + 2.0 ** -39
            assert np.all(np.abs(got[inner] - want_full[inner]) <= bound), (z0, y0, x0)
            continue
        err = np.abs(got[inner] - want_full[inner]).max() / gmax
        assert err <= (TOL64 if mode == "f64" else 3e-6), ((z0, y0, x0), err)


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("mode", ["f64", "f32", "f16s"])
def test_3d_launch_shape_does_not_change_results(q, mode):
    """Rows per wave, tile width, tile order and the wave cap are tuning knobs only: bitwise equal
    states on a ragged lattice (70 columns: a 256-column tile holds two live waves; 7 x 5 rows, so
    row blocks of 2 wide tile rows leave 3 tiles in hardware order)."""
    f = case3(70, 7, 5, 47)
    states = []
    for rows, remap, width, cap, h, st in ((1, 0, 64, 0, 0, 0), (1, 0, 256, 5, 0, 1), (3, 1, 256, 0, 0, 0),
                                           (2, 1, 64, 6, 0, 1), (64, 0, 256, 8, 0, 0), (1, 3, 256, 4, 2, 1),
                                           (1, 3, 64, 0, 1, 0)):
        s, _ = solver3(f, mode, q=q)
        s.set_launch(rows, remap, tile_width=width, max_waves=cap, xcd_rows=h, stores=st)
        s.step(9)
        states.append(s.state_save())
        s.close()
    for st in states[1:]:
        assert torch.equal(st, states[0])


@pytest.mark.parametrize("q", LATTICES)
def test_3d_graph_replay_and_checkpoint(q):
    f = case3(72, 6, 5, 41)
    s, _ = solver3(f, "f32", q=q)
    s.step(3)
    ck = s.state_save()
    s.step(70)
    a = s.populations().cpu().numpy()
    s.state_load(ck, 3)
    for _ in range(70):
        s.step(1)
    b = s.populations().cpu().numpy()
    s.close()
    assert np.array_equal(a, b)


def test_d2q9_d3q19_and_d3q27_share_a_context():
    f = case3(40, 6, 5, 43)
    X, Y, dx = W.mesh(50, 30, -1.0, 1.0)
    p2 = lbm.make_params(50, 30, dx, dx / 4, 0.25, 2e-3, "f64")
    f2 = {"phi0": dev(1 + np.exp(-(X ** 2 + Y ** 2) / 0.1)), "ux": dev(-Y), "uy": dev(X)}
    nz, ny, nx = f["shape"]
    p3 = lbm.make_params(nx, ny, f["dx"], f["dt"], 0.25, f["D_const"], "f64", nz=nz)
    p27 = lbm.make_params(nx, ny, f["dx"], f["dt"], 0.25, f["D_const"], "f32", nz=nz, lattice=27)
    f3 = {"phi0": dev(f["phi0"]), "ux": dev(f["u"][0]), "uy": dev(f["u"][1]), "uz": dev(f["u"][2]), "D": dev(f["D"])}
    insts = ((p2, f2), (p3, f3), (p27, f3))
    both = Solver(list(insts))
    both.step(40)
    got = [both.populations(i).cpu().numpy() for i in range(3)]
    both.close()
    assert got[2].shape == (27, nz, ny, nx)
    for k, (p, ff) in enumerate(insts):
        s = Solver([(p, ff)])
        s.step(40)
        assert np.array_equal(s.populations().cpu().numpy(), got[k])
        s.close()


@pytest.mark.parametrize("q", LATTICES)
def test_3d_errors(q):
    f = case3(8, 5, 4, 1, varD=False)
    nz, ny, nx = f["shape"]
    fields = {"phi0": dev(f["phi0"]), "ux": dev(f["u"][0]), "uy": dev(f["u"][1]), "uz": dev(f["u"][2])}
    mk = lambda **kw: lbm.make_params(nx, ny, f["dx"], f["dt"], 0.25, 2e-3, kw.pop("mode", "f64"), lattice=q, **kw)
    for kw, status in ((dict(nz=nz, aux=lbm.LBM_AUX_FLUX), lbm.LBM_E_UNSUPPORTED),
                       (dict(nz=nz, boundary=lbm.LBM_BC_WALLS), lbm.LBM_E_UNSUPPORTED),
                       (dict(nz=nz, tau3=0.8), lbm.LBM_E_UNSUPPORTED),
                       (dict(nz=2), lbm.LBM_E_ARG)):
        with pytest.raises(lbm.LbmError) as ei:
            Solver([(mk(**kw), fields)])
        assert ei.value.status == status, kw
    with pytest.raises(lbm.LbmError) as ei:
        Solver([(mk(nz=nz), {k: v for k, v in fields.items() if k != "uz"})])
    assert ei.value.status == lbm.LBM_E_ARG
    s = Solver([(mk(nz=nz), fields)])
    with pytest.raises(lbm.LbmError) as ei:
        s.step(1, ux=[fields["ux"]], uy=[fields["uy"]])
    assert ei.value.status == lbm.LBM_E_ARG
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_adjoint_bytes(s.ctx)
    assert ei.value.status == lbm.LBM_E_UNSUPPORTED
    s.close()
