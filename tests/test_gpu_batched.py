"""The batched step (many instances, one launch per step) against serial launches and the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2312_10316_amd import Solver, lbm

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def instance(cfg, mode, aux=lbm.LBM_AUX_LOCAL):
    f = W.rotating_pulse(cfg)
    fields = {k: dev(f[k]) for k in ("phi0", "ux", "uy")}
    if f["D"] is not None:
        fields["D"] = dev(f["D"])
    return lbm.make_params(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, mode, aux), fields, f


def mixed_configs():
    # uneven sizes (ragged 64-column tiles), constant and variable D, different velocities
    return [W.PulseConfig(N=37, U0=2.0, D=3e-3), W.PulseConfig(N=64), W.PulseConfig(N=130, D_variable=True),
            W.PulseConfig(N=3, D=1e-2), W.PulseConfig(N=200, U0=5.0, sigma0=0.15, D_variable=True)]


POLICIES = [(lbm.LBM_BATCH_FLAT, 0, 0), (lbm.LBM_BATCH_STRIDED, 7, 0), (lbm.LBM_BATCH_LPT, 5, 0),
            (lbm.LBM_BATCH_LPT, 4096, 0), (lbm.LBM_BATCH_FLAT, 0, 6), (lbm.LBM_BATCH_LPT, 5, 3)]


@pytest.mark.parametrize("mode", ["f64", "f32", "f16s"])
def test_batched_policies_match_serial_bitwise(mode):
    insts = [instance(c, mode)[:2] for c in mixed_configs()]
    ref = Solver(insts)
    ref.set_batch(lbm.LBM_BATCH_SERIAL)
    ref.step(70)  # two graph replays of 32 steps + 6 eager steps
    want = [ref.state_save(k) for k in range(len(insts))]
    ref.close()
    for policy, blocks, cap in POLICIES:
        s = Solver(insts)
        assert s.get_batch() == {"policy": lbm.LBM_BATCH_FLAT, "blocks": 0,  # default for a uniform batch
                                 "max_waves": 6 if mode == "f32" else 0}
        s.set_batch(policy, blocks, cap)
        s.step(3)
        s.macros()  # synchronizing work between eager steps and graph replays
        s.step(67)
        for k in range(len(insts)):
            assert torch.equal(s.state_save(k), want[k]), (policy, blocks, k)
        s.close()


def test_batched_matches_separate_contexts_and_rows():
    insts = [instance(c, "f32")[:2] for c in mixed_configs()]
    s = Solver(insts)
    s.set_launch(3, 1, inst=2)  # different tile shapes for two instances
    s.set_launch(2, 1, inst=0, tile_width=256)
    for policy, blocks in ((lbm.LBM_BATCH_LPT, 11), (lbm.LBM_BATCH_FLAT, 0)):
        s.set_batch(policy, blocks)
        s.step(20)
    for k, one in enumerate(insts):
        t = Solver([one])
        t.step(40)
        assert torch.equal(t.state_save(), s.state_save(k)), k
        t.close()
    s.close()


def test_batched_fp64_matches_oracle():
    cfgs = [W.PulseConfig(N=48, steps=30, U0=2.5), W.PulseConfig(N=70, steps=30, D_variable=True)]
    built = [instance(c, "f64") for c in cfgs]
    s = Solver([b[:2] for b in built])
    s.set_batch(lbm.LBM_BATCH_LPT, 3)
    s.step(30)
    for k, (cfg, (p, _, f)) in enumerate(zip(cfgs, built)):
        op = O.Problem(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, O.AUX_LOCAL)
        g = O.run(op, O.init(op, f["phi0"], f["ux"], f["uy"]), 30, f["ux"], f["uy"], f["D"])
        got = s.populations(k).cpu().numpy()
        assert np.abs(got - g).max() <= 1e-12 * np.abs(g).max(), k
    s.close()


def test_batched_with_per_instance_sources():
    x1 = W.x1_problem(40, 0.05)
    cfg = W.PulseConfig(N=40)
    f = W.rotating_pulse(cfg)
    pa = lbm.make_params(40, 40, x1["dx"], x1["dt"], x1["lam"], 0.05, "f64")
    pb = lbm.make_params(40, 40, f["dx"], f["dt"], cfg.lam, cfg.D, "f64")
    fa = {k: dev(x1[k]) for k in ("phi0", "ux", "uy")}
    fb = {k: dev(f[k]) for k in ("phi0", "ux", "uy")}
    both = Solver([(pa, fa), (pb, fb)])
    sa, sb = Solver([(pa, fa)]), Solver([(pb, fb)])
    for t in range(x1["steps"]):
        S, dS = x1["source"](t * x1["dt"])
        S, dS = dev(S), dev(dS)
        both.step(1, S=[S, None], dSdt=[dS, None])
        sa.step(1, S=[S], dSdt=[dS])
        sb.step(1)
    assert torch.equal(both.state_save(0), sa.state_save())
    assert torch.equal(both.state_save(1), sb.state_save())
    for s in (both, sa, sb):
        s.close()


def test_mixed_modes_fall_back_to_serial():
    a = instance(W.PulseConfig(N=40), "f64")[:2]
    b = instance(W.PulseConfig(N=40), "f32")[:2]
    s = Solver([a, b])
    assert s.get_batch()["policy"] == lbm.LBM_BATCH_SERIAL
    with pytest.raises(lbm.LbmError) as ei:
        s.set_batch(lbm.LBM_BATCH_FLAT)
    assert ei.value.status == lbm.LBM_E_UNSUPPORTED
    for cap in (2, 9, -1):
        with pytest.raises(lbm.LbmError) as ei:
            s.set_batch(lbm.LBM_BATCH_SERIAL, 0, cap)
        assert ei.value.status == lbm.LBM_E_ARG, cap
    s.step(5)
    t = Solver([b])
    t.step(5)
    assert torch.equal(t.state_save(), s.state_save(1))
    s.close()
    t.close()


def test_seeded_instance_draws_batched():
    """A slice of the seeded 256-instance draw (uneven N, D, U0, sigma0, centre), FP32."""
    draws = W.batched_instances()[:24]
    insts = [instance(d.config, "f32")[:2] for d in draws]
    s = Solver(insts)
    s.set_batch(lbm.LBM_BATCH_LPT, 64)
    s.step(100)
    r = Solver(insts)
    r.set_batch(lbm.LBM_BATCH_SERIAL)
    r.step(100)
    for k in range(len(insts)):
        assert torch.equal(s.state_save(k), r.state_save(k)), k
        st = s.macros(k)
        assert st["nonfinite"] == 0
    s.close()
    r.close()


FUSED_SHAPES = [(128, 16), (256, 4), (512, 1), (128, 37)]


@pytest.mark.parametrize("mode", ["f64", "f32", "f16s", "f16sr"])
def test_batched_two_steps_per_launch_match_serial_single_steps(mode):
    """Every instance of a uniform batch fused (two steps per launch, one batched launch): bitwise the
    serial single steps, for every schedule, tile width and height, at odd and even step counts and
    through graph replays; the single steps of the fused context take the one-step batched kernel."""
    insts = [instance(c, mode)[:2] for c in mixed_configs()]
    ref = Solver(insts)
    ref.set_batch(lbm.LBM_BATCH_SERIAL)
    ref.set_launch(1, 1, tile_width=256)
    ref.step(71)
    want = [ref.state_save(k) for k in range(len(insts))]
    ref.close()
    for (width, rows), (policy, blocks, _) in zip(FUSED_SHAPES * 2, POLICIES[:4] * 2):
        s = Solver(insts)
        s.set_launch(rows, 1, tile_width=width, fuse=2)
        assert all(s.get_launch(k)["fuse"] == 2 for k in range(len(insts)))
        s.set_batch(policy, blocks)
        s.step(3)
        s.macros()
        s.step(68)  # two graph replays of 16 fused launches, then 2 fused launches
        for k in range(len(insts)):
            assert torch.equal(s.state_save(k), want[k]), (mode, width, rows, policy, k)
        s.close()


def test_batched_two_steps_per_launch_rejections():
    insts = [instance(c, "f32")[:2] for c in mixed_configs()]
    s = Solver(insts)
    with pytest.raises(lbm.LbmError) as ei:
        s.set_launch(16, 1, inst=0, tile_width=128, fuse=2)  # one instance of several: all or none
    assert ei.value.status == lbm.LBM_E_ARG
    s.close()
    mixed = [instance(mixed_configs()[0], "f32")[:2], instance(mixed_configs()[1], "f64")[:2]]
    s = Solver(mixed)  # not a uniform batch
    with pytest.raises(lbm.LbmError) as ei:
        s.set_launch(16, 1, tile_width=128, fuse=2)
    assert ei.value.status == lbm.LBM_E_ARG
    s.close()
