"""lbm_macros_static (the variant of lbm_macros that allocates nothing: its reduction scratch is a
static device array) against lbm_macros on the same states, through the C ABI, on two calls in a row,
the second on a smaller lattice, plus a call on a third context after both."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2312_10316_amd import Solver, lbm

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def context(n, mode, steps, lattice=None):
    if lattice is None:
        cfg = W.PulseConfig(N=n, steps=steps, D_variable=True)
        f = W.rotating_pulse(cfg)
        p = lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode)
        s = Solver([(p, {k: dev(f[k]) for k in ("phi0", "ux", "uy", "D")})])
        ref = dev(W.pulse_reference(cfg, f))
    else:
        cfg = W.PulseConfig(N=n, steps=steps)
        f = W.rotating_pulse3(cfg)
        p = lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode, nz=n, lattice=lattice)
        s = Solver([(p, {"phi0": dev(f["phi0"]), "ux": dev(f["u"][0]), "uy": dev(f["u"][1]), "uz": dev(f["u"][2])})])
        ref = dev(W.pulse3_reference(cfg, f))
    s.step(steps)
    return s, ref


def both(s, ref):
    shape = ref.shape
    pa = torch.empty(shape, dtype=torch.float64, device="cuda")
    pb = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    a = lbm.lbm_macros(s.ctx, 0, pa, ref)
    b = lbm.lbm_macros_static(s.ctx, 0, pb, ref)
    return a, b, pa, pb


@pytest.mark.parametrize("mode", ["f64", "f32", "f16s"])
def test_static_scratch_macros_equal_workspace_macros(mode):
    for n, steps in ((1536, 37), (96, 5)):  # the second call on a smaller lattice (fewer reduction blocks)
        s, ref = context(n, mode, steps)
        a, b, pa, pb = both(s, ref)
        assert a == b, (n, a, b)  # every statistic bitwise, the step counter and status included
        assert torch.equal(pa, pb)
        b2 = lbm.lbm_macros_static(s.ctx, 0, None, None)
        a2 = lbm.lbm_macros(s.ctx, 0, None, None)
        assert a2 == b2
        s.close()
    s, ref = context(24, "f64", 7, lattice=19)  # a 3D lattice afterwards
    a, b, pa, pb = both(s, ref)
    assert a == b and torch.equal(pa, pb)
    s.close()


def test_static_scratch_macros_report_blow_up_and_bad_calls():
    s, ref = context(64, "f64", 3)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_macros_static(s.ctx, 1, None, None)
    assert ei.value.status == lbm.LBM_E_STATE
    assert lbm.lib().lbm_macros_static(s.ctx, 0, None, None, None) == lbm.LBM_E_ARG
    s.close()
    X, Y, dx = W.mesh(40, 30, -1.0, 1.0)
    phi0 = np.exp(-(X ** 2 + Y ** 2))
    phi0[3, 4] = np.nan
    p = lbm.make_params(40, 30, dx, dx / 4, 0.25, 1e-3, "f64")
    s = Solver([(p, {"phi0": dev(phi0), "ux": dev(0 * X), "uy": dev(0 * X)})])
    a = lbm.lbm_macros(s.ctx, 0, None, None, raise_nonfinite=False)
    b = lbm.lbm_macros_static(s.ctx, 0, None, None, raise_nonfinite=False)
    assert a["status"] == b["status"] == lbm.LBM_E_NONFINITE and a["nonfinite"] == b["nonfinite"] >= 1
    s.close()
