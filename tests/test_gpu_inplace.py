"""One-buffer (in-place) stepping.  A single periodic instance updates one population buffer in place
(the AA pattern: a streaming step and a local step alternate): D3Q19/D3Q27 instances whose two buffers
would not fit in the 256 MiB Infinity Cache but whose one buffer does by default, D2Q9 instances on
request (lbm_set_launch stores = 2; their default is two steps per launch on two buffers).  States are
compared bitwise with the same instance advanced on two buffers: the reference context holds a second,
small instance, which keeps it on two buffers, and runs one launch per instance."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2312_10316_amd import Solver, lbm

pytestmark = pytest.mark.gpu

# (mode, nx, ny, variable D): two buffers touch 278-280 MB per step, one buffer 153-165 MB
CASES = [("f32", 2048, 1700, False, 0.0), ("f32", 2048, 1700, True, 0.0), ("f16s", 2048, 3100, False, 0.0),
         ("f64", 1024, 1700, False, 0.0), ("f32", 2048, 1700, False, 0.8),  # MRT-R, tau3 = 0.8
         ("f64", 1024, 1700, True, 0.8)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def instance(mode, nx, ny, var, tau3=0.0, aux=lbm.LBM_AUX_LOCAL):
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    fields = {"phi0": dev(1.0 + np.exp(-((X - 0.3) ** 2 + Y ** 2) / 0.05)), "ux": dev(-np.pi * Y), "uy": dev(np.pi * X)}
    if var:
        fields["D"] = dev(1e-3 * (1.0 + 0.5 * np.sin(np.pi * X) * np.sin(np.pi * Y)))
    return lbm.make_params(nx, ny, dx, dx / 10, 0.25, 1e-3, mode, aux, phi_ref=1.0, tau3=tau3), fields


def pair(mode, nx, ny, var, tau3=0.0, aux=lbm.LBM_AUX_LOCAL):
    p, fields = instance(mode, nx, ny, var, tau3, aux)
    one = Solver([(p, fields)])
    one.set_launch(1, 1, tile_width=256, stores=2)
    small = instance(mode, 64, 40, False, tau3, aux)
    two = Solver([(p, fields), small])
    two.set_batch(lbm.LBM_BATCH_SERIAL)
    return one, two


@pytest.mark.parametrize("mode,nx,ny,var,tau3", CASES)
def test_in_place_matches_two_buffers(mode, nx, ny, var, tau3):
    one, two = pair(mode, nx, ny, var, tau3)
    assert one.get_launch()["stores"] == 2 and two.get_launch()["stores"] != 2
    for n in (1, 1, 5, 70, 3):  # odd and even counts; 70 replays a captured graph of 64 steps
        one.step(n)
        two.step(n)
        assert torch.equal(one.populations(), two.populations(0)), n
        a, b = one.macros(), two.macros(0)
        assert a["mass"] == b["mass"] and a["step"] == b["step"], n
    one.close()
    two.close()


def test_in_place_state_images_and_restrictions():
    """State images are the two-buffer ones at any step (converted after an odd count), load at either
    parity, and move between the one- and two-buffer contexts."""
    one, two = pair(*CASES[0])
    one.step(3)
    two.step(3)
    img = one.state_save()
    assert torch.equal(img, two.state_save(0))  # odd step: converted to the standard image
    one.step(1)                                 # the other parity ...
    one.state_load(img, 3)                      # ... takes the same image
    one.step(2)
    two.step(2)
    assert torch.equal(one.populations(), two.populations(0))
    assert torch.equal(one.state_save(), two.state_save(0))
    two.step(1)
    one.state_load(two.state_save(0), 6)        # a two-buffer image into the one-buffer context (odd parity)
    one.step(3)
    two.step(3)
    assert torch.equal(one.state_save(), two.state_save(0))
    assert one.macros()["step"] == two.macros(0)["step"] == 9
    for kw in (dict(stores=2, rows=2), dict(stores=2, fuse=2, tile_width=256)):
        with pytest.raises(lbm.LbmError) as ei:
            one.set_launch(kw.pop("rows", 1), 1, **dict(dict(tile_width=256), **kw))
        assert ei.value.status == lbm.LBM_E_ARG, kw
    # switching between one buffer and two at either parity carries the state over
    for stores, n in ((0, 3), (2, 1), (1, 2), (2, 2), (0, 1)):
        one.set_launch(1, 1, tile_width=256, stores=stores)
        assert one.get_launch()["stores"] == stores
        one.step(n)
        two.step(n)
        assert torch.equal(one.state_save(), two.state_save(0)), (stores, n)
    one.set_launch(1, 3, tile_width=256, max_waves=5, xcd_rows=4, stores=2)  # launch shape: still bitwise
    one.step(3)
    two.step(3)
    assert torch.equal(one.populations(), two.populations(0))
    with pytest.raises(lbm.LbmError) as ei:
        two.set_launch(1, 1, tile_width=256, stores=2)
    assert ei.value.status == lbm.LBM_E_ARG
    assert lbm.lbm_adjoint_bytes(one.ctx, 0) > 0  # the adjoint works on images, so it is available
    X, Y, _ = W.mesh(CASES[0][1], CASES[0][2], -1.0, 1.0)  # a new velocity field after an odd step count
    ux2, uy2 = dev(-2.0 * Y), dev(2.0 * X)
    one.step(1)
    two.step(1)
    one.set_velocity(ux2, uy2)
    two.set_velocity(ux2, uy2, inst=0)
    one.step(65)
    two.step(65)
    assert torch.equal(one.state_save(), two.state_save(0))
    one.close()
    two.close()


@pytest.mark.parametrize("aux", [lbm.LBM_AUX_LOCAL, lbm.LBM_AUX_NONE])
def test_in_place_with_a_source(aux):
    """The source path (a time-dependent S and dS/dt every step) and the form without the auxiliary
    term, in place and on two buffers: bitwise equal."""
    one, two = pair("f32", 2048, 1700, False, 0.0, aux)
    assert one.get_launch()["stores"] == 2
    X, Y, _ = W.mesh(2048, 1700, -1.0, 1.0)
    base = np.exp(-(X ** 2 + Y ** 2) / 0.1)
    for t in range(5):
        S, dS = dev(np.cos(0.3 * t) * base), dev(-0.3 * np.sin(0.3 * t) * base)
        one.step(1, S=[S], dSdt=[dS])
        two.step(1, S=[S, None], dSdt=[dS, None])
        assert torch.equal(one.populations(), two.populations(0)), t
    one.close()
    two.close()


# (velocities, mode, n): n^3 lattices where one population buffer fits in the cache and two do not
CASES3 = [(19, "f32", 128), (27, "f32", 112), (27, "f16s", 140), (19, "f64s_f32m", 104)]


def instance3(q, mode, n):
    X, Y, Z, dx = W.mesh3(n, n, n, -1.0, 1.0)
    fields = {"phi0": dev(1.0 + np.exp(-((X - 0.3) ** 2 + Y ** 2 + Z ** 2) / 0.05)), "ux": dev(-np.pi * Y),
              "uy": dev(np.pi * X), "uz": dev(0.1 * np.sin(np.pi * Z))}
    return lbm.make_params(n, n, dx, dx / 10, 0.25, 1e-3, mode, phi_ref=1.0, nz=n, lattice=q), fields


@pytest.mark.parametrize("q,mode,n", CASES3)
def test_3d_in_place_matches_two_buffers(q, mode, n):
    p, fields = instance3(q, mode, n)
    one = Solver([(p, fields)])
    two = Solver([(p, fields), instance3(q, mode, 12)])
    assert one.get_launch()["stores"] == 2 and two.get_launch()["stores"] != 2
    for k in (1, 2, 70):  # steps 1, 3 (odd) and 73 (odd, through graph replays)
        one.step(k)
        two.step(k)
        assert torch.equal(one.state_save(), two.state_save(0)), k
    one.step(1)
    two.step(1)
    assert torch.equal(one.populations(), two.populations(0))
    img = two.state_save(0)
    one.step(1)                 # odd parity: the image is converted on load
    one.state_load(img, 74)
    one.step(3)
    two.step(3)
    assert torch.equal(one.state_save(), two.state_save(0))
    a, b = one.macros(), two.macros(0)
    assert a["mass"] == b["mass"]
    one.close()
    two.close()


def test_3d_fp64_math_keeps_two_buffers():
    """With FP64 math the one-row in-place 3D kernels would round the collision differently from the
    two-buffer walking loop (the compiler fuses its multiply-adds otherwise), so such an instance keeps
    two buffers even where only one fits."""
    p, fields = instance3(19, "f64", 104)
    s = Solver([(p, fields)])
    assert s.get_launch()["stores"] == 0
    s.close()
