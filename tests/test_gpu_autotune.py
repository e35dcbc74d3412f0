"""The launch autotuner on the GPU: it times candidates on the caller's instances without
advancing them (states and step counters restored bitwise), applies the winner, and caches it."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2312_10316_amd import Solver, autotune, lbm

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def pulse_instance(n, mode="f32", seed=0):
    cfg = W.PulseConfig(N=n, steps=10, U0=2.0 + 0.1 * seed)
    f = W.rotating_pulse(cfg)
    p = lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode)
    return p, {k: dev(f[k]) for k in ("phi0", "ux", "uy")}


def states(s):
    return [s.populations(k).cpu().numpy() for k in range(len(s.params))]


@pytest.mark.parametrize("multi", [False, True])
def test_tuning_does_not_advance_and_results_do_not_depend_on_the_winner(multi, tmp_path):
    inst = [pulse_instance(n, seed=k) for k, n in enumerate((96, 130, 64, 200))] if multi else [pulse_instance(160)]
    s = Solver(inst)
    s.step(7)
    before = states(s)
    cands = [(1, 1, 0, 64, 0, 0, lbm.LBM_BATCH_SERIAL, 0), (2, 0, 0, 256, 5, 1, lbm.LBM_BATCH_SERIAL, 0),
             (1, 3, 2, 256, 5, 0, lbm.LBM_BATCH_SERIAL, 0)]
    if not multi:  # one instance also tries two steps per launch and one buffer in place
        cands += [(16, 1, 0, 256, 0, 0, lbm.LBM_BATCH_SERIAL, 0, 2), (8, 0, 0, 128, 0, 1, lbm.LBM_BATCH_SERIAL, 0, 2),
                  (1, 1, 0, 256, 0, 2, lbm.LBM_BATCH_SERIAL, 0, 1)]
    if multi:
        cands += [(1, 1, 0, 256, 0, 1, lbm.LBM_BATCH_FLAT, 0), (1, 1, 0, 64, 0, 0, lbm.LBM_BATCH_LPT, 512),
                  (2, 1, 0, 256, 0, 1, lbm.LBM_BATCH_STRIDED, 256), (1, 1, 0, 256, 0, 0, lbm.LBM_BATCH_LPT, 512)]
    cache = str(tmp_path / "tune.json")
    r = autotune.tune(s, cands, steps=16, reps=1, cache_path=cache, force=True)
    assert tuple(r["best"]) in [tuple(c) for c in cands] and not r["cached"]
    assert all(np.array_equal(a, b) for a, b in zip(before, states(s)))
    assert all(s.macros(k)["step"] == 7 for k in range(len(inst)))
    rows, remap, h, width, cap, stores, policy, blocks, fuse = (tuple(r["best"]) + (1,))[:9]
    assert s.get_launch(0) == {"rows": rows, "xcd_remap": remap, "tile_width": width, "max_waves": cap,
                               "xcd_rows": h, "stores": stores, "fuse": fuse}
    s.step(20)
    tuned = states(s)
    s.close()
    ref = Solver(inst)
    ref.step(27)
    assert all(np.array_equal(a, b) for a, b in zip(tuned, states(ref)))
    ref.close()
    again = Solver(inst)
    r2 = autotune.tune(again, cands, steps=16, reps=1, cache_path=cache)
    assert r2["cached"] and r2["best"] == r["best"]
    again.close()


def test_tuning_a_d3q19_instance():
    X, Y, Z, dx = W.mesh3(70, 20, 12, -1.0, 1.0)
    p = lbm.make_params(70, 20, dx, dx / 4, 0.25, 2e-3, "f32", nz=12)
    f = {"phi0": dev(1 + np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 0.1)), "ux": dev(-Y), "uy": dev(X), "uz": dev(0 * X)}
    s = Solver([(p, f)])
    before = states(s)
    r = autotune.tune(s, [(1, 0, 0, 64, 0, 0, 0, 0), (1, 1, 0, 256, 5, 1, 0, 0), (2, 1, 0, 256, 0, 0, 0, 0),
                          (1, 3, 4, 256, 4, 1, 0, 0)], steps=8, reps=1, force=True)
    assert all(np.array_equal(a, b) for a, b in zip(before, states(s)))
    assert s.get_launch(0)["rows"] == r["best"][0]
    s.close()


def test_default_candidates_of_a_single_instance_include_fused_and_in_place_launches():
    s = Solver([pulse_instance(128)])
    cands = autotune.default_candidates(s)
    assert any(c[8] == 2 for c in cands) and any(c[5] == 2 for c in cands)
    s.close()
    s = Solver([pulse_instance(64), pulse_instance(96)])  # a uniform batch: fused candidates as a whole
    cands = autotune.default_candidates(s)
    assert any(c[8] == 1 for c in cands) and any(c[8] == 2 for c in cands)
    assert all(c[6] in (lbm.LBM_BATCH_FLAT, lbm.LBM_BATCH_LPT) and c[3] in (128, 256) for c in cands if c[8] == 2)
    s.close()
