"""Two steps per launch (temporal blocking, lbm_launch.fuse = 2) against single steps and the oracle.

A fused launch computes each block's intermediate state (its tile plus a one-node frame) in LDS and
writes only the state two steps later.  Every node goes through the same per-node arithmetic and
the intermediate populations through the storage codec, so fused contexts must be bitwise equal to
one-step contexts, whatever the tile width, tile height, tile order and store kind, at odd and even
step counts (an odd count ends with a single step)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2312_10316_amd import Solver, lbm

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def case(nx, ny, seed, var=True):
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    rng = np.random.default_rng(seed)
    c = 4.0
    ux = c * (0.25 * np.sin(np.pi * Y + rng.uniform(0, 6)) - 0.1 * Y)
    uy = c * (0.2 * np.cos(np.pi * X + rng.uniform(0, 6)) + 0.15 * X)
    phi0 = 0.3 + np.exp(-((X - 0.2) ** 2 + (Y + 0.1) ** 2) / 0.1) + 0.05 * rng.uniform(0, 1, (ny, nx))
    f = dict(phi0=phi0, ux=ux, uy=uy)
    if var:
        f["D"] = 2e-3 * (1 + 0.5 * rng.uniform(-1, 1, (ny, nx)))
    return dx, dx / c, f


def contexts(mode, nx, ny, seed, aux=lbm.LBM_AUX_LOCAL, var=True, tau3=0.0, shape=(256, 16, 1, 0, 1)):
    dx, dt, f = case(nx, ny, seed, var)
    p = lbm.make_params(nx, ny, dx, dt, 0.25, 2e-3, mode, aux, phi_ref=0.3, tau3=tau3)
    fields = {k: dev(v) for k, v in f.items()}
    one = Solver([(p, fields)])
    one.set_launch(1, 1, tile_width=256, stores=0)
    two = Solver([(p, fields)])
    width, rows, remap, h, stores = shape
    two.set_launch(rows, remap, tile_width=width, xcd_rows=h, stores=stores, fuse=2)
    return one, two, (p, f, dx, dt)


SHAPES = [(256, 16, 1, 0, 1), (128, 3, 0, 0, 0), (512, 1, 2, 0, 1), (256, 64, 3, 2, 0), (128, 7, 3, 1, 1),
          (512, 256, 1, 0, 0)]


@pytest.mark.parametrize("mode", ["f64", "f64s_f32m", "f32", "f16s", "f16sr"])
@pytest.mark.parametrize("nx,ny", [(70, 45), (130, 67), (3, 3), (64, 5), (300, 7), (513, 130)])
def test_fused_equals_single_steps(mode, nx, ny):
    for k, shape in enumerate(SHAPES[:3] if nx * ny < 1000 else SHAPES):
        one, two, _ = contexts(mode, nx, ny, seed=nx + ny + k, shape=shape)
        assert two.get_launch()["fuse"] == 2
        for n in (2, 1, 5, 70, 4):  # even and odd counts; 70 replays a graph of 16 fused launches
            one.step(n)
            two.step(n)
            assert torch.equal(one.state_save(), two.state_save()), (shape, n)
        a, b = one.macros(), two.macros()
        assert a["mass"] == b["mass"] and a["step"] == b["step"] == 82
        one.close()
        two.close()


@pytest.mark.parametrize("aux,var,tau3", [(lbm.LBM_AUX_NONE, True, 0.0), (lbm.LBM_AUX_LOCAL, False, 0.0),
                                          (lbm.LBM_AUX_LOCAL, True, 1.0), (lbm.LBM_AUX_NONE, False, 0.0)])
@pytest.mark.parametrize("mode", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("shape", [(256, 8, 1, 0, 0), (512, 40, 1, 0, 0)])
def test_fused_variants_equal_single_steps(mode, aux, var, tau3, shape):
    """No auxiliary term, constant D, tau3 = 1 (TRT-R written as MRT-R), and a per-call source; on
    512-column tiles 42 walk rows (FP16 storage there computes the frame nodes 32 rows at a time)."""
    one, two, (p, f, dx, dt) = contexts(mode, 200, 90, seed=11, aux=aux, var=var, tau3=tau3, shape=shape)
    rng = np.random.default_rng(5)
    S = dev(0.05 * rng.uniform(-1, 1, (90, 200)))
    for n, src in ((4, True), (3, False), (6, True)):
        kw = dict(S=[S], dSdt=[S * -0.5]) if src else {}
        one.step(n, **kw)
        two.step(n, **kw)
        assert torch.equal(one.state_save(), two.state_save()), n
    one.close()
    two.close()


def test_fused_fp64_matches_the_oracle():
    nx, ny, steps = 70, 45, 26
    one, two, (p, f, dx, dt) = contexts("f64", nx, ny, seed=3, shape=(128, 5, 0, 0, 0))
    two.step(steps)
    op = O.Problem(nx, ny, dx, dt, 0.25, 2e-3, O.AUX_LOCAL)
    g = O.run(op, O.init(op, f["phi0"], f["ux"], f["uy"]), steps, f["ux"], f["uy"], f["D"])
    got = two.populations().cpu().numpy()
    assert np.abs(got - g).max() <= 1e-12 * np.abs(g).max()
    one.close()
    two.close()


@pytest.mark.parametrize("mode,n", [("f32", 2048), ("f16s", 2048), ("f64", 2048), ("f32", 8192), ("f16s", 8192),
                                    ("f16sr", 8192)])
def test_fused_full_size_equals_single_steps(mode, n):
    """The benchmark's lattice sizes in the fused default shape: four steps, bitwise."""
    cfg = W.PulseConfig(N=n, steps=4, D_variable=(n == 8192))
    f = W.rotating_pulse(cfg)
    keys = ("phi0", "ux", "uy", "D") if cfg.D_variable else ("phi0", "ux", "uy")
    fields = {k: dev(f[k]) for k in keys}
    p = lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode)
    print(f"fused full size: {mode} {n}^2", flush=True)
    one = Solver([(p, fields)])
    one.set_launch(1, 1, tile_width=256, stores=0)
    one.step(4)
    ref = one.state_save()
    one.close()
    two = Solver([(p, fields)])
    two.set_launch(32, 1, tile_width=256, stores=0, fuse=2)
    two.step(4)
    assert torch.equal(two.state_save(), ref)
    two.close()


def test_fused_rejects_what_it_does_not_cover():
    dx, dt, f = case(64, 40, 1)
    fields = {k: dev(v) for k, v in f.items()}

    def mk(**kw):
        return lbm.make_params(64, 40, dx, dt, 0.25, 2e-3, "f32", **kw)

    for params, inst, width in (([mk(boundary=lbm.LBM_BC_NEE)], -1, 256), ([mk(boundary=lbm.LBM_BC_WALLS)], -1, 256),
                                ([mk(), mk()], 1, 256), ([mk(), mk(tau3=0.7)], -1, 256), ([mk(tau3=0.7)], -1, 256),
                                ([mk(aux=lbm.LBM_AUX_FLUX)], -1, 512),
                                ([mk(aux=lbm.LBM_AUX_FLUX), mk(aux=lbm.LBM_AUX_FLUX)], -1, 256)):
        s = Solver([(p, fields) for p in params])
        with pytest.raises(lbm.LbmError) as ei:
            s.set_launch(8, 1, inst=inst, tile_width=width, fuse=2)
        assert ei.value.status == lbm.LBM_E_ARG
        s.close()
    s = Solver([(mk(), fields)])
    for kw in (dict(tile_width=64), dict(tile_width=1024), dict(rows=0), dict(rows=257), dict(max_waves=5),
               dict(stores=2), dict(fuse=3)):
        args = dict(rows=8, xcd_remap=1, tile_width=256, fuse=2)
        args.update(kw)
        with pytest.raises(lbm.LbmError) as ei:
            s.set_launch(args.pop("rows"), args.pop("xcd_remap"), **args)
        assert ei.value.status == lbm.LBM_E_ARG, kw
    s.close()


FLUX_SHAPES = [(256, 16, 1, 0, 1), (128, 3, 0, 0, 0), (256, 1, 2, 0, 0), (128, 64, 3, 2, 1)]


@pytest.mark.parametrize("mode", ["f64", "f64s_f32m", "f32", "f16s", "f16sr"])
@pytest.mark.parametrize("nx,ny", [(70, 45), (3, 3), (64, 5), (300, 7), (513, 130), (130, 4)])
def test_fused_flux_form_equals_single_steps(mode, nx, ny):
    """The flux form's two-step tiles (three frame columns each side, phi rings at both levels):
    bitwise the one-step flux kernel, for four tile shapes, at odd and even step counts."""
    for k, shape in enumerate(FLUX_SHAPES[:2] if nx * ny < 1000 else FLUX_SHAPES):
        one, two, _ = contexts(mode, nx, ny, seed=nx + ny + k, aux=lbm.LBM_AUX_FLUX, shape=shape)
        for n in (2, 1, 5, 70, 4):
            one.step(n)
            two.step(n)
            assert torch.equal(one.state_save(), two.state_save()), (shape, n)
        one.close()
        two.close()


@pytest.mark.parametrize("var,tau3,src", [(False, 0.0, False), (True, 1.0, True), (False, 0.0, True)])
@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_fused_flux_form_variants(mode, var, tau3, src):
    """Constant D, tau3 = 1 (TRT-R written as MRT-R) and a per-call source in the flux form."""
    one, two, (p, f, dx, dt) = contexts(mode, 200, 90, seed=17, aux=lbm.LBM_AUX_FLUX, var=var, tau3=tau3,
                                        shape=(256, 8, 1, 0, 0))
    rng = np.random.default_rng(7)
    S = dev(0.05 * rng.uniform(-1, 1, (90, 200)))
    for n in (4, 3, 6):
        kw = dict(S=[S], dSdt=[S * 0.25]) if src else {}
        one.step(n, **kw)
        two.step(n, **kw)
        assert torch.equal(one.state_save(), two.state_save()), n
    one.close()
    two.close()


def test_fused_flux_form_fp64_matches_the_oracle():
    nx, ny, steps = 70, 45, 26
    one, two, (p, f, dx, dt) = contexts("f64", nx, ny, seed=5, aux=lbm.LBM_AUX_FLUX, shape=(128, 5, 0, 0, 0))
    two.step(steps)
    op = O.Problem(nx, ny, dx, dt, 0.25, 2e-3, O.AUX_FLUX)
    g = O.run(op, O.init(op, f["phi0"], f["ux"], f["uy"]), steps, f["ux"], f["uy"], f["D"])
    got = two.populations().cpu().numpy()
    assert np.abs(got - g).max() <= 1e-12 * np.abs(g).max()
    one.close()
    two.close()


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_fused_flux_form_full_size_equals_single_steps(mode):
    """8192^2 with D(x) in the flux form's default two-step shape: four steps, bitwise."""
    n = 8192
    cfg = W.PulseConfig(N=n, steps=4, D_variable=True)
    f = W.rotating_pulse(cfg)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy", "D")}
    p = lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode, lbm.LBM_AUX_FLUX)
    print(f"fused flux full size: {mode} {n}^2", flush=True)
    one = Solver([(p, fields)])
    one.set_launch(2, 1, tile_width=256, stores=0)
    one.step(4)
    ref = one.state_save()
    one.close()
    two = Solver([(p, fields)])
    assert two.get_launch()["fuse"] == 2
    two.step(4)
    assert torch.equal(two.state_save(), ref)
    two.close()
