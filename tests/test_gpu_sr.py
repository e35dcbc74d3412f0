"""FP16 storage with stochastic rounding (LBM_STORE_F16SR) through the C ABI, against the oracle.

The oracle's rounding (``oracle/rounding.py``, pinned on the CPU) and its own SplitMix64 stream decide
every code from the same FP32 value.  Where the GPU forms that value exactly as numpy does (the initial
state with u = 0: FP32 products w_i phi0), the codes must be bitwise equal.  After a step the GPU's
FP32 collision differs from the oracle's FP64 one by a few FP32 units, so a decision is compared
wherever the oracle's distance to the rounding threshold exceeds a band of 64 / 2^13 of the FP16
spacing; those decisions must all agree, and every code must be one of the two FP16 neighbours of the
oracle's value.  Launch shapes, two steps per launch, one buffer in place, graph replays, batches and
checkpoints must not change a single code (the random bits depend only on node, time level and seed).
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import rounding as R
from paper_2312_10316_amd import Solver, lbm

pytestmark = pytest.mark.gpu

K = 15  # scale_log2
BAND = 64


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def codes(s, p, inst=0):
    """The stored FP16 codes of the state image as [ny, 9, nx] (slot i of node x)."""
    raw = s.state_save(inst).cpu().numpy().view(np.float16)
    pitch = lbm.pitch_of(p)
    return raw[:p.ny * 9 * pitch].reshape(p.ny, 9, pitch)[:, :, :p.nx]


def wrefs(phi_ref):
    _, _, w = O.lattice()
    return np.asarray(w) * phi_ref


@pytest.mark.parametrize("phi_ref,seed,tiny", [(0.0, 0, False), (0.5, 12345, False), (0.0, -1, False),
                                               (0.0, 77, True)])
def test_initial_codes_are_the_oracle_rounding(phi_ref, seed, tiny):
    """u = 0: g_eq_i = w_i phi0 in FP32, rounded stochastically at time level 0 with the bits of the
    node that computed it; bitwise equal to the oracle's rounding of the same FP32 value.  `tiny` puts
    phi0 at +-10^-14 .. 10^-4 (and some exact zeros), so that many codes are FP16 subnormals."""
    nx, ny = 300, 200
    rng = np.random.default_rng(31)
    phi0 = rng.uniform(-1.0, 3.0, (ny, nx))
    if tiny:
        phi0 = rng.choice([-1.0, 1.0], (ny, nx)) * 10.0 ** rng.uniform(-14, -4, (ny, nx))
        phi0[::7, ::5] = 0.0
    z = np.zeros((ny, nx))
    p = lbm.make_params(nx, ny, 1.0, 1.0, 0.25, 1e-3, "f16sr", scale_log2=K, phi_ref=phi_ref, round_seed=seed)
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(z), "uy": dev(z)})])
    img = codes(s, p)
    s.close()
    ex, ey, w = O.lattice()
    r = R.node_random_ints(seed & 0xFFFFFFFF, nx * ny, np.arange(nx * ny).reshape(ny, nx), 0)
    p32 = phi0.astype(np.float32)
    differs = 0
    for i in range(9):
        v = (np.float32(w[i]) * p32 - np.float32(w[i] * phi_ref)) * np.float32(2.0 ** K)
        want = R.f16_round_stochastic(v, r[..., i])
        got = np.roll(img[:, i, :], (int(ey[i]), int(ex[i])), (0, 1))  # slot i of node x - e_i
        assert np.array_equal(got.view(np.uint16), want.view(np.uint16)), i
        differs += int((want != R.f16_round_nearest(v)).sum())
        if tiny:
            assert (np.abs(want.astype(np.float64)) < 2.0 ** -14).mean() > 0.3  # subnormal codes
    assert differs > 0.15 * 9 * nx * ny  # a quarter of the codes differ from round-to-nearest


def test_fp16_subnormal_codes_round_to_nearest():
    """The deterministic code on FP16 subnormals: bitwise numpy's round-to-nearest-even."""
    nx, ny = 300, 200
    rng = np.random.default_rng(37)
    phi0 = rng.choice([-1.0, 1.0], (ny, nx)) * 10.0 ** rng.uniform(-14, -4, (ny, nx))
    z = np.zeros((ny, nx))
    p = lbm.make_params(nx, ny, 1.0, 1.0, 0.25, 1e-3, "f16s", scale_log2=K)
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(z), "uy": dev(z)})])
    img = codes(s, p)
    s.close()
    ex, ey, w = O.lattice()
    p32 = phi0.astype(np.float32)
    for i in range(9):
        v = (np.float32(w[i]) * p32 - np.float32(0.0)) * np.float32(2.0 ** K)
        got = np.roll(img[:, i, :], (int(ey[i]), int(ex[i])), (0, 1))
        assert np.array_equal(got.view(np.uint16), R.f16_round_nearest(v).view(np.uint16)), i


def _case(nx, ny, seed):
    X, Y, dx = W.mesh(nx, ny, -1.0, 1.0)
    rng = np.random.default_rng(seed)
    c = 4.0
    ux = c * (0.25 * np.sin(np.pi * Y + rng.uniform(0, 6)) - 0.1 * Y)
    uy = c * (0.2 * np.cos(np.pi * X + rng.uniform(0, 6)) + 0.15 * X)
    phi0 = 0.3 + np.exp(-((X - 0.2) ** 2 + (Y + 0.1) ** 2) / 0.1) + 0.05 * rng.uniform(0, 1, (ny, nx))
    D = 2e-3 * (1 + 0.5 * rng.uniform(-1, 1, (ny, nx)))
    return dx, dx / c, dict(phi0=phi0, ux=ux, uy=uy, D=D)


def _check_decisions(img, g_new, p, phi_ref, seed, level):
    """img: GPU codes [ny, 9, nx] of P_i(x) at `level`; g_new: the oracle's pre-collision state one step
    later (P_i(x) streamed to x + e_i, periodic).  A decision is clear where the oracle's value lies
    farther than eps from the rounding threshold and from both FP16 neighbours, eps being the larger
    of BAND / 2^13 of the FP16 spacing and 2^-19 w_i max|phi| 2^K (the FP32 collision's absolute
    error: P_i is w_i times a sum of magnitude phi, rounded a few times in FP32, 2^-24 each).  A wrong
    random bit, node or time level would flip about half of the clear decisions."""
    ex, ey, w = O.lattice()
    nx, ny = p.nx, p.ny
    r = R.node_random_ints(seed & 0xFFFFFFFF, nx * ny, np.arange(nx * ny).reshape(ny, nx), level)
    wr = wrefs(phi_ref)
    phimax = float(np.abs(O.phi(O.Problem(nx, ny, 1.0, 1.0, 0.25), g_new)).max())
    checked = total = 0
    for i in range(9):
        P = np.roll(g_new[i], (-int(ey[i]), -int(ex[i])), (0, 1))  # P_i at its own node
        v = R.f16s_value(P[None], wr[i:i + 1], K)[0]
        a = np.abs(v.astype(np.float64))
        lo, ulp = R.f16_floor_neighbours(a)
        eps = np.maximum(BAND * ulp / 2 ** 13, 2.0 ** -19 * w[i] * phimax * 2.0 ** K)
        thr = lo + r[..., i] * ulp / 2 ** 13
        got = img[:, i, :].astype(np.float64)
        # every code is an FP16 neighbour of the oracle's value, up to the FP32 error
        assert np.all(np.abs(np.abs(got) - a) <= 2 * ulp + eps)
        clear = (np.abs(a - thr) > eps) & (a - lo > eps) & (lo + ulp - a > eps)
        assert np.all(np.abs(np.abs(got[clear]) - a[clear]) < ulp[clear])
        want = R.f16_round_stochastic(v, r[..., i]).astype(np.float64)
        assert np.array_equal(got[clear], want[clear]), (i, int((got[clear] != want[clear]).sum()))
        checked += int(clear.sum())
        total += clear.size
    print(f"decisions checked: {checked} of {total}")
    assert checked > 0.5 * total


@pytest.mark.parametrize("aux,tau3", [(lbm.LBM_AUX_LOCAL, 0.0), (lbm.LBM_AUX_FLUX, 0.0), (lbm.LBM_AUX_NONE, 0.0),
                                      (lbm.LBM_AUX_LOCAL, 0.7)])
def test_step_decisions_match_the_oracle(aux, tau3):
    """70 steps in the default launch (graph replays), then one more; the codes of that step against the
    oracle stepping the GPU state (two steps per launch meet these codes bitwise in test_gpu_fused)."""
    nx, ny, seed, phi_ref = 70, 45, 7, 0.3
    dx, dt, f = _case(nx, ny, 3)
    p = lbm.make_params(nx, ny, dx, dt, 0.25, 2e-3, "f16sr", aux, scale_log2=K, phi_ref=phi_ref, tau3=tau3,
                        round_seed=seed)
    s = Solver([(p, {k: dev(v) for k, v in f.items()})])
    s.step(70)
    g0 = s.populations().cpu().numpy()
    s.step(1)
    img = codes(s, p)
    assert s.macros()["step"] == 71
    s.close()
    op = O.Problem(nx, ny, dx, dt, 0.25, 2e-3, aux, tau3=tau3)
    g1 = O.step(op, g0, f["ux"], f["uy"], f["D"])
    _check_decisions(img, g1, p, phi_ref, seed, 71)


def _pair(nx, ny, seed=5, **kw):
    dx, dt, f = _case(nx, ny, 11)
    p = lbm.make_params(nx, ny, dx, dt, 0.25, 2e-3, "f16sr", scale_log2=K, phi_ref=0.3, round_seed=seed, **kw)
    fields = {k: dev(v) for k, v in f.items()}
    return p, Solver([(p, fields)]), Solver([(p, fields)])


@pytest.mark.parametrize("shape", [(256, 16, 1, 0, 1), (128, 3, 0, 0, 0), (512, 5, 3, 2, 0)])
def test_two_steps_per_launch_and_launch_shapes_are_bitwise(shape):
    p, one, two = _pair(200, 130)
    one.set_launch(1, 1, tile_width=256, stores=0)
    width, rows, remap, h, stores = shape
    two.set_launch(rows, remap, tile_width=width, xcd_rows=h, stores=stores, fuse=2)
    for n in (2, 1, 5, 70, 4):
        one.step(n)
        two.step(n)
        assert torch.equal(one.state_save(), two.state_save()), (shape, n)
    one.set_launch(4, 3, tile_width=64, xcd_rows=1, max_waves=5)
    two.set_launch(1, 1, tile_width=256, stores=2)  # one buffer in place
    for n in (3, 66, 2):
        one.step(n)
        two.step(n)
        assert torch.equal(one.state_save(), two.state_save()), n
    one.close()
    two.close()


@pytest.mark.parametrize("shape", [(256, 24, 1, 0, 0), (256, 7, 3, 1, 0), (512, 16, 1, 0, 1)])
def test_two_steps_per_launch_constant_D_is_bitwise(shape):
    """Without a D field: on 256-column tiles with streaming stores the fused walk computes its frame
    nodes four rows at a time (on 512-column tiles in step with the walk); bitwise the single steps."""
    dx, dt, f = _case(300, 130, 12)
    p = lbm.make_params(300, 130, dx, dt, 0.25, 2e-3, "f16sr", scale_log2=K, phi_ref=0.3, round_seed=9)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy")}
    one, two = Solver([(p, fields)]), Solver([(p, fields)])
    one.set_launch(1, 1, tile_width=256, stores=0)
    width, rows, remap, h, stores = shape
    two.set_launch(rows, remap, tile_width=width, xcd_rows=h, stores=stores, fuse=2)
    for n in (2, 1, 5, 70, 4):
        one.step(n)
        two.step(n)
        assert torch.equal(one.state_save(), two.state_save()), (shape, n)
    one.close()
    two.close()


def test_checkpoint_resume_needs_the_step_count():
    p, a, b = _pair(96, 64)
    a.step(33)
    img = a.state_save()
    a.step(40)
    b.state_load(img, 33)
    b.step(40)
    assert torch.equal(a.state_save(), b.state_save())
    b.state_load(img, 34)  # the same state at another time level draws other bits
    b.step(40)
    assert not torch.equal(a.state_save(), b.state_save())
    a.close()
    b.close()


def test_seeds_and_batches():
    """Instances with different seeds in one batched launch equal separate contexts bitwise; another
    seed gives other codes."""
    dx, dt, f = _case(90, 70, 13)
    fields = {k: dev(v) for k, v in f.items()}
    ps = [lbm.make_params(90, 70, dx, dt, 0.25, 2e-3, "f16sr", scale_log2=K, phi_ref=0.3, round_seed=sd)
          for sd in (1, 2, 3)]
    batch = Solver([(p, fields) for p in ps])
    assert batch.get_batch()["policy"] != lbm.LBM_BATCH_SERIAL
    batch.step(67)
    for k, p in enumerate(ps):
        s = Solver([(p, fields)])
        s.step(67)
        assert torch.equal(s.state_save(), batch.state_save(k)), k
        s.close()
    assert not torch.equal(batch.state_save(0), batch.state_save(1))
    batch.close()


def test_rejected_where_not_built():
    z = dev(np.zeros((8, 8, 8)))
    p3 = lbm.make_params(8, 8, 1.0, 1.0, 0.25, 1e-3, "f16sr", nz=8)
    with pytest.raises(lbm.LbmError) as ei:
        Solver([(p3, {"phi0": z, "ux": z, "uy": z, "uz": z})])
    assert ei.value.status == lbm.LBM_E_UNSUPPORTED
    z2 = dev(np.zeros((8, 8)))
    p = lbm.make_params(8, 8, 1.0, 1.0, 0.25, 1e-3, "f16s", round_seed=3)
    with pytest.raises(lbm.LbmError) as ei:
        Solver([(p, {"phi0": z2, "ux": z2, "uy": z2})])
    assert ei.value.status == lbm.LBM_E_ARG
