"""Throughput of the TRT-R D2Q9 step on one MI355X: MLUPS and fraction of the HBM roofline.

A "step" is one time step of the whole hot path (one fused pull-stream-collide launch per step)
over the full lattice.  Default workload: the rotating Gaussian pulse on a periodic 2048^2 lattice
(c = dx/dt = 10, U0 = pi, D = 1e-3, Lambda = 1/4), warmup + timed steps = 3200 (t = 0.3125).
The headline `value` is FP32 storage; FP64, FP64-storage/FP32-math and shifted FP16 storage are
timed on the same workload and reported under "modes" with their errors against the closed form and
against the FP64 path.

    python bench.py [--gpus 1] [--steps 3000] [--warmup 200] [--n 2048] [--modes f32,f64,f64s_f32m,f16s]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q9 TRT-R MLUPS & % HBM roofline, FP32/FP16 vs FP64 at fixed L2 error"
HBM_PEAK_GBPS = 8000.0
STORE_BYTES = {"f64": 8, "f64s_f32m": 8, "f32": 4, "f16s": 2, "f16sr": 2}
FIELD_BYTES = {"f64": 8, "f64s_f32m": 4, "f32": 4, "f16s": 4, "f16sr": 4}
KERNEL_SRC = os.path.join(ROOT, "paper_2312_10316_amd", "csrc", "lbm_kernels.hip")


def bytes_per_lup(mode: str, variable_D: bool) -> int:
    """Algorithmic HBM bytes per lattice update: 9 populations read + 9 written, u (2 components),
    D when it is a field."""
    return 18 * STORE_BYTES[mode] + 2 * FIELD_BYTES[mode] + (FIELD_BYTES[mode] if variable_D else 0)


def launch_bytes_per_lup(mode: str, variable_D: bool, launch: dict) -> float:
    """Algorithmic bytes per lattice update of the launch that ran: a launch of two fused steps reads
    the state and the fields once and writes the state once for two updates of every node."""
    return bytes_per_lup(mode, variable_D) / max(int(launch.get("fuse", 1) or 1), 1)


def roofline_bound(stores: int) -> str:
    """What bounds a step by where its state lives: streamed to HBM (non-temporal stores, lbm_launch
    stores 0), or held in the 256 MiB Infinity Cache (cached stores 1, one buffer in place 2)."""
    return "hbm" if stores == 0 else "infinity_cache"


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in ("lbm_kernels.hip", "lbm_fused.hip", "lbm_kernel_common.h", "lbm_device.h", "lbm_internal.h",
                 "lbm_api.hip"):
        with open(os.path.join(ROOT, "paper_2312_10316_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(mode: str, n: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_hash():
        return None
    e = d.get("entries", {}).get(f"{mode}_{n}")
    return None if e is None else e.get("bytes_per_launch")


def run_mode(mode, n, steps, warmup, torch, W, lbm, Solver, graph=True):
    cfg = W.PulseConfig(N=n, steps=warmup + steps)
    f = W.rotating_pulse(cfg)
    dev = {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy")}
    p = lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode)
    stream = torch.cuda.current_stream()
    s = Solver([(p, dev)], stream=stream)
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ref = torch.from_numpy(W.pulse_reference(cfg, f)).cuda()
    st, phi = s.macros(ref=ref, want_phi=True)
    launch = s.get_launch()
    s.close()
    lups = float(n) * n * steps
    return {
        "mlups": lups / (ms * 1e-3) / 1e6,
        "ms_per_step": ms / steps,
        "E_r": st["rms_err"],
        "L2_rel": st["l2_rel_err"],
        "max_err": st["max_abs_err"],
        "mass": st["mass"],
        "nonfinite": st["nonfinite"],
        "t_end": cfg.t_end,
        "launch": launch,
    }, phi


def run_batched(torch, W, lbm, Solver, n_inst=256, steps=2000, eager_steps=100):
    """The seeded batch of uneven pulse instances (FP32): aggregate MLUPS of serial per-instance
    launches (eager, and graph-replayed) against the autotuned single-launch batched step.  The
    batched figure is one run of exactly `steps` steps from the initial state; after it every
    instance's phi is checked (finite or not) and measured against its closed form."""
    import numpy as np

    from paper_2312_10316_amd import autotune
    draws = W.batched_instances(n_inst, steps=steps)
    insts, refs = [], []
    for d in draws:
        cfg = d.config
        f = W.rotating_pulse(cfg)
        p = lbm.make_params(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, "f32")
        insts.append((p, {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy")}))
        refs.append(torch.from_numpy(W.pulse_reference(cfg, f)).cuda())
    sizes = np.array([d.N * d.N for d in draws], dtype=np.float64)
    nodes = float(sizes.sum())
    s = Solver(insts)
    init = [s.state_save(k) for k in range(n_inst)]

    def timed(fn, nsteps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        fn()
        e1.record(s.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / nsteps

    out = {"instances": n_inst, "nodes": int(nodes), "steps": steps, "storage": "f32",
           "sizes": f"N log-uniform in [32, 512], seed 231210316 (min {min(d.N for d in draws)}, "
                    f"max {max(d.N for d in draws)})"}
    s.set_batch(lbm.LBM_BATCH_SERIAL)
    # serial baselines: one launch per instance and step in the one-step shape of a batch (two steps per
    # launch of a small lattice is a latency-bound walk of few blocks, far slower one instance at a time)
    s.set_launch(1, 1, tile_width=64)
    s.step(2)

    def eager():
        for _ in range(eager_steps):
            s.step(1)
    ms = timed(eager, eager_steps)
    out["serial_eager"] = {"ms_per_step": ms, "mlups": nodes / (ms * 1e-3) / 1e6}
    s.step(64)
    ms = timed(lambda: s.step(steps), steps)
    out["serial_graph"] = {"ms_per_step": ms, "mlups": nodes / (ms * 1e-3) / 1e6}
    t = autotune.tune(s, steps=64, reps=2)
    s.step(64)  # captures the graphs of the tuned launch
    for k in range(n_inst):
        s.state_load(init[k], 0, inst=k)
    ms = timed(lambda: s.step(steps), steps)
    out["batched"] = {"ms_per_step": ms, "mlups": nodes / (ms * 1e-3) / 1e6,
                      "config": {"rows": t["best"][0], "xcd_remap": t["best"][1], "xcd_rows": t["best"][2],
                                 "tile_width": t["best"][3], "max_waves": t["best"][4], "stores": t["best"][5],
                                 "policy": ["serial", "flat", "strided", "lpt"][t["best"][6]], "blocks": t["best"][7],
                                 "fuse": t["best"][8]}}
    # the tuner's best one-step and best two-step candidates (ms per step while tuning)
    by_fuse = {}
    for cand, t_ms in t["ms_per_step"].items():
        fz = json.loads(cand)[8] if len(json.loads(cand)) > 8 else 1
        by_fuse[fz] = min(by_fuse.get(fz, float("inf")), t_ms)
    out["tuning"] = {f"best_{'two' if fz == 2 else 'one'}_step_launch": {"ms_per_step": v, "mlups": nodes / (v * 1e-3) / 1e6}
                     for fz, v in sorted(by_fuse.items())}
    out["speedup_vs_serial_graph"] = out["serial_graph"]["ms_per_step"] / ms
    out["speedup_vs_serial_eager"] = out["serial_eager"]["ms_per_step"] / ms
    stats = [s.macros(k, ref=refs[k], raise_nonfinite=False) for k in range(n_inst)]
    s.close()
    finite = np.array([st["nonfinite"] == 0 and st["step"] == steps for st in stats])
    # bounded: finite and within twice the initial peak (the closed form never exceeds 1, the pulse's
    # initial peak); finite instances above that are on their way to blowing up
    peak = np.array([st["max_abs_phi"] for st in stats])
    bounded = finite & (peak <= 2.0)
    er = np.array([st["rms_err"] for st in stats])
    tau1 = np.array([0.5 + 3.0 * d.D * d.config.dt / d.config.dx ** 2 for d in draws])
    umax = np.array([d.U0 * math.sqrt(2.0) / d.config.c for d in draws])  # corner |u| / c
    bins = [0.0, 0.003, 0.01, 0.03, 0.1, 1.0]
    by_tau = []
    for lo, hi in zip(bins[:-1], bins[1:]):
        m = (tau1 - 0.5 >= lo) & (tau1 - 0.5 < hi)
        by_tau.append({"tau1_minus_half": [lo, hi], "instances": int(m.sum()), "bounded": int((m & bounded).sum()),
                       "unbounded_finite": int((m & finite & ~bounded).sum()), "nonfinite": int((m & ~finite).sum())})
    out["accuracy"] = {
        "criterion": "bounded = every phi finite and max|phi| <= 2 after the run (the closed form stays <= 1)",
        "bounded_instances": int(bounded.sum()), "unbounded_finite_instances": int((finite & ~bounded).sum()),
        "nonfinite_instances": int((~finite).sum()),
        "E_r_bounded": {"min": float(er[bounded].min()), "median": float(np.median(er[bounded])),
                        "max": float(er[bounded].max())} if bounded.any() else None,
        "E_r_per_instance": [float(e) if ok else None for e, ok in zip(er, bounded)],
        "by_tau1": by_tau,
        "bounded_u_over_c_max": float(umax[bounded].max()) if bounded.any() else None,
        "unstable_u_over_c_min": float(umax[~bounded].min()) if (~bounded).any() else None,
    }
    out["batched"]["mlups_bounded_instances"] = float(sizes[bounded].sum()) / (ms * 1e-3) / 1e6
    return out


def _timed_steps(torch, s, nsteps):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(nsteps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / max(nsteps, 1)


def run_hbm(torch, W, lbm, Solver, n=8192, steps=200, warmup=32, modes=("f32", "f16s", "f16sr", "f64", "f64s_f32m")):
    """The streaming regime: the rotating pulse (constant D) on a periodic n^2 lattice whose two
    population buffers (1.2-9.7 GB at 8192^2) far exceed the 256 MiB Infinity Cache, so every step
    reads and writes HBM.  Per storage mode: MLUPS over `steps` graph-replayed steps (HIP events on
    the launch stream) and the algorithmic bytes per second against the 8 TB/s HBM peak."""
    cfg = W.PulseConfig(N=n, steps=steps + warmup)
    f = W.rotating_pulse(cfg)
    dev = {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy")}
    out = {"workload": f"rotating Gaussian pulse, periodic {n}^2, c=10, U0=pi, D=1e-3 (constant), "
                       f"{warmup}+{steps} steps", "N": n}
    for mode in modes:
        s = Solver([(lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode), dev)])
        s.step(warmup)
        ms = _timed_steps(torch, s, steps)
        launch = s.get_launch()
        s.close()
        bpl = launch_bytes_per_lup(mode, False, launch)
        mlups = n * n / (ms * 1e-3) / 1e6
        achieved = mlups * bpl / 1e3
        traffic = traffic_from_profile(mode, n)
        out[mode] = {"mlups": mlups, "ms_per_step": ms, "bytes_per_lup": bpl, "achieved_gbps": achieved,
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None if traffic is None else round(traffic),
                     "launch": launch}
        print(f"# hbm {n}^2 {mode}: {mlups:.0f} MLUPS, {achieved:.0f} GB/s ({achieved / HBM_PEAK_GBPS:.3f})",
              file=sys.stderr, flush=True)
    del dev
    torch.cuda.empty_cache()
    return out


def run_precision_8192(torch, W, lbm, Solver, n=8192, steps=1000):
    """8192^2, D(x) = 1e-3 (1 + 0.5 sin(pi x) sin(pi y)), 1000 steps: every storage mode, errors of
    phi against the FP64 run, mass drift."""
    cfg = W.PulseConfig(N=n, steps=steps, D_variable=True)
    f = W.rotating_pulse(cfg)
    dev = {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy", "D")}
    out, ref = {}, None
    for mode in ("f64", "f64s_f32m", "f32", "f16s", "f16sr"):
        s = Solver([(lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode), dev)])
        m0 = s.macros()["mass"]
        s.step(64)
        ms = _timed_steps(torch, s, steps - 64)
        st, phi = s.macros(want_phi=True, raise_nonfinite=False)
        launch = s.get_launch()
        s.close()
        bpl = launch_bytes_per_lup(mode, True, launch)
        r = {"mlups": n * n / (ms * 1e-3) / 1e6, "ms_per_step": ms,
             "hbm_gbps_algorithmic": n * n / (ms * 1e-3) * bpl / 1e9,
             "bytes_per_lup": bpl, "mass_drift": st["mass"] / m0 - 1.0,
             "nonfinite": st["nonfinite"], "fuse": launch["fuse"]}
        if mode == "f64":
            ref = phi
        else:
            d = (phi - ref).abs()
            r["max_err_vs_f64"] = float(d.max())
            r["l2_rel_err_vs_f64"] = float(torch.sqrt((d * d).sum() / (ref * ref).sum()))
            del d
        r["roofline_frac"] = r["hbm_gbps_algorithmic"] / HBM_PEAK_GBPS
        out[mode] = r
        del phi
    # offset pulse: phi0 + 1 on a background of 1 with the FP16 shift phi_ref = 1 (the stored codes
    # carry g - w_i, so the background costs no precision); errors of phi - 1 against the FP64 run
    dev["phi0"] = dev["phi0"] + 1.0
    s = Solver([(lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, "f16s", phi_ref=1.0), dev)])
    s.step(steps)
    st, phi = s.macros(want_phi=True, raise_nonfinite=False)
    s.close()
    d = (phi - 1.0 - ref).abs()
    out["f16s_offset_phi_ref_1"] = {"max_err_vs_f64": float(d.max()),
                                    "l2_rel_err_vs_f64": float(torch.sqrt((d * d).sum() / (ref * ref).sum())),
                                    "nonfinite": st["nonfinite"]}
    del d, phi, ref, dev
    torch.cuda.empty_cache()
    return out


def run_refinement(torch, W, lbm, Solver, sizes=(64, 128, 256, 512, 1024, 2048),
                   modes=("f64", "f32", "f16s", "f16sr")):
    """E_r against the closed-form pulse at t = 0.3125 under acoustic (c = 10) and diffusive
    (dx^2/dt fixed at its 256^2 value) refinement; least-squares orders over N >= 256 (the coarse grids
    under-resolve sigma0 = 0.1); N* = finest N at which a reduced-precision mode stays within 5 % of the
    FP64 E_r; with acoustic scaling also each mode's MLUPS per N (400 more steps, timed after the
    error is read) and its speedup over FP64 at N*, i.e. at equal error against the closed form."""
    import numpy as np
    out = {}
    for scaling in ("acoustic", "diffusive"):
        res = {m: [] for m in modes}
        mlups = {m: [] for m in modes}
        for N in sizes:
            cfg = W.refinement(N, scaling)
            f = W.rotating_pulse(cfg)
            dev = {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy")}
            ref = torch.from_numpy(W.pulse_reference(cfg, f)).cuda()
            for m in modes:
                s = Solver([(lbm.make_params(N, N, f["dx"], cfg.dt, cfg.lam, cfg.D, m), dev)])
                s.step(cfg.steps)
                res[m].append(s.macros(ref=ref, raise_nonfinite=False)["rms_err"])
                if scaling == "acoustic":
                    mlups[m].append(N * N / (_timed_steps(torch, s, 400) * 1e-3) / 1e6)
                s.close()
        entry = {"N": list(sizes), "E_r": res}
        if scaling == "acoustic":
            entry["mlups"] = mlups
        for m in modes:
            e = np.array(res[m])
            ok = np.isfinite(e) & (e > 0) & (np.array(sizes) >= 256)
            entry.setdefault("order", {})[m] = (float(-np.polyfit(np.log(np.array(sizes)[ok]), np.log(e[ok]), 1)[0])
                                                if ok.sum() >= 2 else None)
            if m != "f64":
                within = [N for N, a, b in zip(sizes, res[m], res["f64"]) if np.isfinite(a) and a <= 1.05 * b]
                entry.setdefault("N_star", {})[m] = max(within) if within else None
                if within and scaling == "acoustic":
                    k = list(sizes).index(max(within))
                    entry.setdefault("speedup_at_N_star", {})[m] = mlups[m][k] / mlups["f64"][k]
        out[scaling] = entry
    return out


def run_flux(torch, W, lbm, Solver, sizes=((2048, 3000), (8192, 200))):
    """The flux form of the aux term (default launch: two steps per launch) at 2048^2 and 8192^2, FP32 and
    FP64: MLUPS, the launch's algorithmic bytes per second against 8 TB/s, and the single-step-equivalent
    rate (the bytes a one-step launch would move for the same updates)."""
    out = {}
    for n, steps in sizes:
        cfg = W.PulseConfig(N=n, steps=steps)
        f = W.rotating_pulse(cfg)
        dev = {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy")}
        for mode in ("f32", "f64"):
            s = Solver([(lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode, lbm.LBM_AUX_FLUX), dev)])
            s.step(64)
            ms = _timed_steps(torch, s, steps)
            launch = s.get_launch()
            s.close()
            mlups = n * n / (ms * 1e-3) / 1e6
            bpl = launch_bytes_per_lup(mode, False, launch)
            key = mode if n == 2048 else f"{mode}_{n}"
            out[key] = {"N": n, "mlups": mlups, "ms_per_step": ms, "launch": launch, "bytes_per_lup": bpl,
                        "frac": mlups * bpl / 1e3 / HBM_PEAK_GBPS,
                        "single_step_equivalent_frac": mlups * bytes_per_lup(mode, False) / 1e3 / HBM_PEAK_GBPS}
        del dev
        torch.cuda.empty_cache()
    return out


def run_dirichlet(torch, W, lbm, Solver, sizes=(100, 200, 400, 800), kappa=0.05, n_tp=2048, tp_steps=2000):
    """The Sec. 3 benchmark on its own (N+1)^2 grid with Dirichlet edges by non-equilibrium
    extrapolation: E_r at t = 1 (Table 2 extended past N = 100) per storage mode, with S, dS/dt and
    the Dirichlet values of the closed form supplied every step; and the throughput of the
    Dirichlet-edge step kernel at (n_tp+1)^2 (graph-replayed, S and phi_b held fixed)."""
    import numpy as np
    out = {"kappa": kappa, "N": list(sizes), "E_r": {}, "order": {}}
    for mode in ("f64", "f32", "f16s", "f16sr"):
        errs = []
        for N in sizes:
            x1 = W.x1_problem(N, kappa, dirichlet=True)
            n = x1["nx"]
            dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
            p = lbm.make_params(n, n, x1["dx"], x1["dt"], x1["lam"], kappa, mode, lbm.LBM_AUX_LOCAL,
                                boundary=lbm.LBM_BC_NEE)
            s = Solver([(p, {k: dv(x1[k]) for k in ("phi0", "ux", "uy")})])
            S0 = dv(x1["source"](0.0)[0])
            q_exact0 = dv(x1["exact"](0.0))
            for k in range(x1["steps"]):  # S(t), phi(t) decay as exp(-2 kappa t) from their t = 0 forms
                a = math.exp(-2.0 * kappa * k * x1["dt"])
                s.set_dirichlet(q_exact0 * a)
                S = S0 * a
                s.step(1, S=[S], dSdt=[S * (-2.0 * kappa)])
            T = x1["steps"] * x1["dt"]
            ref = q_exact0 * math.exp(-2.0 * kappa * T)
            s.set_dirichlet(ref)
            errs.append(s.macros(ref=ref)["rms_err"])
            s.close()
        out["E_r"][mode] = errs
        out["order"][mode] = [None] + [math.log(errs[k - 1] / errs[k]) / math.log(sizes[k] / sizes[k - 1])
                                       for k in range(1, len(sizes))]
    x1 = W.x1_problem(n_tp, kappa, dirichlet=True)
    n = x1["nx"]
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    S, dS = (dv(a) for a in x1["source"](0.0))
    tp = {}
    for mode in ("f32", "f64"):
        for bc in (lbm.LBM_BC_NEE, lbm.LBM_BC_PERIODIC):
            p = lbm.make_params(n, n, x1["dx"], x1["dt"], x1["lam"], kappa, mode, lbm.LBM_AUX_LOCAL, boundary=bc)
            s = Solver([(p, {k: dv(x1[k]) for k in ("phi0", "ux", "uy")})])
            s.step(64, S=[S], dSdt=[dS])
            ms = _timed_steps(torch, s, tp_steps)
            s.close()
            tp[f"{mode}_{'nee' if bc == lbm.LBM_BC_NEE else 'periodic'}"] = {
                "mlups": n * n / (ms * 1e-3) / 1e6, "ms_per_step": ms}
    out["throughput"] = {"nodes": f"{n}^2", "with_source": True, **tp}
    return out


def run_3d(torch, W, lbm, Solver, q=19, sizes=(64, 128, 256), tp_steps=400):
    """Rotating pulse about the z axis on [-1, 1]^3 (c = 10, D = 1e-3, t = 0.3125) on the D3Q19 or
    D3Q27 lattice: E_r against the closed form per storage mode and size, the step's throughput at the
    largest size, and at the size before it (128^3: its state fits in the Infinity Cache, with cached
    stores or one buffer updated in place, so that rate is not bound by HBM)."""
    import numpy as np
    BYTES = {"f64": q * 16 + 24, "f64s_f32m": q * 16 + 12, "f32": q * 8 + 12, "f16s": q * 4 + 12}
    out = {"N": list(sizes), "E_r": {m: [] for m in BYTES}, "throughput": {}, "throughput_cache": {}}
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for n in sizes:
        cfg = W.PulseConfig(N=n, steps=int(round(0.3125 / (2.0 / n / 10.0))))
        f = W.rotating_pulse3(cfg)
        fields = {"phi0": dv(f["phi0"]), "ux": dv(f["u"][0]), "uy": dv(f["u"][1]), "uz": dv(f["u"][2])}
        ref = dv(W.pulse3_reference(cfg, f))
        mk = lambda mode: lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode, nz=n, lattice=q)
        for mode in BYTES:
            s = Solver([(mk(mode), fields)])
            if n == sizes[-1] or (len(sizes) > 1 and n == sizes[-2]):
                stores = s.get_launch()["stores"]
                s.step(64)
                ms = _timed_steps(torch, s, tp_steps)
                s.close()
                s = Solver([(mk(mode), fields)])
                mlups = n ** 3 / (ms * 1e-3) / 1e6
                key = "throughput" if n == sizes[-1] else "throughput_cache"
                out[key][mode] = {"mlups": mlups, "ms_per_step": ms, "bytes_per_lup": BYTES[mode],
                                  "hbm_gbps_algorithmic": mlups * BYTES[mode] / 1e3,
                                  "roofline_frac": mlups * BYTES[mode] / 1e3 / HBM_PEAK_GBPS,
                                  "stores": ["non-temporal", "cached", "one buffer in place"][stores]}
            s.step(cfg.steps)
            out["E_r"][mode].append(s.macros(ref=ref)["rms_err"])
            s.close()
        del fields, ref
        torch.cuda.empty_cache()
    out["nodes"] = f"{sizes[-1]}^3"
    if len(sizes) > 1:
        out["nodes_cache"] = f"{sizes[-2]}^3"
    return out


def run_adjoint(torch, W, lbm, Solver):
    """512^2 pulse, 400 steps, FP32 forward with sqrt(T) checkpoints; D on a 32 x 32 bicubic control
    grid; loss = 1/2 sum (phi_T - phi_target)^2 against the run with D = 1e-3.  The context is created
    by a first forward/backward pass; the second pass (same D) is timed: the forward (checkpoints
    included) and the backward (per segment: recomputation and adjoint steps in one library call)."""
    from paper_2312_10316_amd import adjoint
    cfg = W.PulseConfig(N=W.C5_N, steps=W.C5_STEPS)
    f = W.rotating_pulse(cfg)
    dv = lambda a: torch.from_numpy(a).cuda()
    mk = lambda mode: adjoint.RunSpec(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, dv(f["phi0"]), dv(f["ux"]),
                                      dv(f["uy"]), cfg.steps, mode)
    B = adjoint.bspline_operator(cfg.N, W.C5_CTRL)
    tspec = mk("f32")
    with torch.no_grad():
        target = adjoint.simulate(torch.full((cfg.N, cfg.N), cfg.D, dtype=torch.float64, device="cuda"), tspec)
    tspec.close()
    spec = mk("f32")
    out = {"N": cfg.N, "steps": cfg.steps, "control_grid": W.C5_CTRL}
    for rep in range(2):
        theta = dv(W.control_theta(W.C5_CTRL)).requires_grad_(True)
        D = adjoint.D_from_control(theta, B, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi = adjoint.simulate(D, spec)
        loss = 0.5 * ((phi - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    spec.close()
    lups = float(cfg.N) ** 2 * cfg.steps
    out.update(checkpoints=spec.stats["checkpoints"], segment=spec.stats["segment"],
               forward_s=t1 - t0, backward_s=t2 - t1, backward_over_forward=(t2 - t1) / (t1 - t0),
               forward_mlups=lups / (t1 - t0) / 1e6, adjoint_mlups=lups / (t2 - t1) / 1e6,
               loss=float(loss.detach()), grad_norm=float(theta.grad.norm()),
               note="timed on the second forward/backward pass of one context (the first creates it); "
                    "adjoint MLUPS = N^2 x steps / backward seconds, the backward doing one recomputed "
                    "forward step and one adjoint step per step")
    return out


def run_tau2_sweep(torch, W, lbm, Solver, tau1=0.8, tau2s=(1.0, 1.1, 1.2, 1.3, 1.375, 1.45, 1.5, 1.6, 1.7, 1.8)):
    """Sec. 3.3: steady diffusion with a uniform source across a channel between halfway
    anti-bounce-back walls (x periodic, u = 0, FP64): relative RMS error of the converged profile
    against the exact linear-plus-parabolic one, over the free relaxation time tau2 at tau1 = 0.8.
    The paper's slip-free relation puts the minimum at tau2 = 3(1 - 4 tau1)/(8(1 - 2 tau1)) = 1.375."""
    import numpy as np
    nx, ny, lo, hi, S0 = 64, 24, 0.3, 0.7, 2e-3
    kappa = (tau1 - 0.5) / 3.0
    y = np.arange(ny)[:, None] + 0.5
    exact = lo + (hi - lo) * y / ny + S0 / (2 * kappa) * y * (ny - y)
    z = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    pb = torch.full((ny, nx), 0.5, dtype=torch.float64, device="cuda")
    pb[0, :], pb[-1, :] = lo, hi
    S = torch.full((ny, nx), S0, dtype=torch.float64, device="cuda")
    errs, steps_used = [], []
    for tau2 in tau2s:
        p = lbm.make_params(nx, ny, 1.0, 1.0, (tau1 - 0.5) * (tau2 - 0.5), kappa, "f64", lbm.LBM_AUX_LOCAL,
                            boundary=lbm.LBM_BC_WALLS)
        s = Solver([(p, {"phi0": torch.full((ny, nx), 0.5, dtype=torch.float64, device="cuda"), "ux": z, "uy": z})])
        s.set_dirichlet(pb)
        prev, n = None, 0
        while n < 400000:
            s.step(4096, S=[S])
            n += 4096
            _, phi = s.macros(want_phi=True)
            phi = phi.cpu().numpy()
            if prev is not None and np.abs(phi - prev).max() < 1e-15:
                break
            prev = phi
        s.close()
        errs.append(float(np.sqrt(np.mean((phi - exact) ** 2)) / np.abs(exact).max()))
        steps_used.append(n)
    k = int(np.argmin(errs))
    return {"tau1": tau1, "tau2": list(tau2s), "relative_rms_error": errs, "steps_to_converge": steps_used,
            "argmin_tau2": tau2s[k], "slip_free_tau2_theory": 3 * (1 - 4 * tau1) / (8 * (1 - 2 * tau1)),
            "channel": f"{nx} x {ny} lattice units, walls at y = -1/2 and {ny} - 1/2, values {lo} and {hi}, "
                       f"uniform source {S0}"}


def copy_bandwidth(torch, lbm, nbytes=2 << 30, reps=20, cached=False):
    """Read + write bandwidth of the library's plain copy kernel, one pass per call: by default the
    streaming (non-temporal) copy of 2 GiB, which calibrates HBM; with ``cached`` the default-policy
    copy, which on buffers that together fit in the 256 MiB Infinity Cache calibrates a step whose
    state stays in that cache."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    fn = lbm.lbm_bench_copy_cached if cached else lbm.lbm_bench_copy
    for _ in range(5):
        fn(b, a)
        fn(a, b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn(b, a)
        fn(a, b)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * 2 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def cpu_host() -> dict:
    """The host the oracle is timed on: core counts and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "model": model,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def _oracle_threads(host) -> int:
    """Threads of the all-cores leg: OMP_NUM_THREADS when set (the host's share), else every usable CPU."""
    env = host.get("omp_num_threads_env")
    return int(env) if env and env.isdigit() and int(env) > 0 else int(host["usable_cpus"] or 1)


def cpu_baseline(n, budget_s=12.0, cross_check=True, cross_budget_s=150.0):
    """The FP64 oracle as it stands (plain C, gcc -O2 -ffp-contract=off), timed on this host's cores:
    single-threaded and with its OpenMP build over all cores (bitwise the same results), on bounded
    samples of the benchmark workload and on the workloads the oracle is run on in full: the 64^2
    parity pulse, the Sec. 3 benchmark at N = 100, the 256^2 and 512^2 refinement members, and the
    1024^2 x 1000-step variable-D cross-check of the precision study.  Returns (json, the oracle's phi
    of the cross-check or None)."""
    import numpy as np

    import oracle as O
    import workloads as W
    host = cpu_host()
    threads = _oracle_threads(host)
    legs = []

    def pulse_problem(cfg):
        f = W.rotating_pulse(cfg)
        p = O.Problem(cfg.N, cfg.N, f["dx"], cfg.dt, cfg.lam, cfg.D, O.AUX_LOCAL)
        return f, p, O.init(p, f["phi0"], f["ux"], f["uy"])

    def timed_run(cfg, nsteps, nthreads):
        f, p, g = pulse_problem(cfg)
        t0 = time.perf_counter()
        if nthreads == 1:
            g = O.run(p, g, nsteps, f["ux"], f["uy"], D=f["D"])
            used = 1
        else:
            g, used = O.run_threads(p, g, nsteps, f["ux"], f["uy"], D=f["D"], threads=nthreads)
        el = time.perf_counter() - t0
        return g, p, f, el, used

    # the benchmark workload (2048^2 pulse), bounded samples: one thread, then all cores
    cfg = W.PulseConfig(N=n, steps=3200)
    probe = max(1, int(round(2.0e6 / (n * n)))) if n <= 1024 else 1
    _, _, _, el, _ = timed_run(cfg, probe, 1)
    k1 = max(1, min(3200, int(budget_s / max(el / probe, 1e-9))))
    _, _, _, el1, _ = timed_run(cfg, k1, 1)
    single = {"value": n * n * k1 / el1 / 1e6, "threads": 1, "steps": k1, "seconds": el1}
    kt = max(1, min(3200, int(budget_s * threads / max(el / probe, 1e-9) / 2)))
    _, _, _, elt, used = timed_run(cfg, kt, threads)
    allc = {"value": n * n * kt / elt / 1e6, "threads": used, "steps": kt, "seconds": elt}

    # workloads run in full
    c1 = W.PulseConfig(N=64, steps=160)
    g, p, f, el, used = timed_run(c1, c1.steps, 1)
    legs.append({"workload": "64^2 rotating pulse, 160 steps (t = 0.5)", "threads": used, "seconds": el,
                 "mlups": 64 * 64 * 160 / el / 1e6,
                 "E_r": O.rms_error(O.phi(p, g), W.pulse_reference(c1, f))})
    x1 = W.x1_problem(100, 0.05)
    p = O.Problem(100, 100, x1["dx"], x1["dt"], x1["lam"], 0.05, O.AUX_LOCAL)
    g = O.init(p, x1["phi0"], x1["ux"], x1["uy"])
    t0 = time.perf_counter()
    for k in range(x1["steps"]):
        S, dS = x1["source"](k * x1["dt"])
        g = O.step(p, g, x1["ux"], x1["uy"], None, S, dS)
    el = time.perf_counter() - t0
    legs.append({"workload": "Sec. 3 benchmark, periodic proxy N = 100, kappa = 0.05, t = 1 (100 steps, "
                             "per-step source)", "threads": 1, "seconds": el,
                 "mlups": 100 * 100 * x1["steps"] / el / 1e6,
                 "E_r_times_N_over_N_plus_1": O.rms_error(O.phi(p, g), x1["exact"](x1["steps"] * x1["dt"])) * 100 / 101,
                 "table2_printed": 5.984e-4})
    for N in (256, 512):
        cfg = W.refinement(N, "acoustic")
        g, p, f, el, used = timed_run(cfg, cfg.steps, threads)
        legs.append({"workload": f"{N}^2 rotating pulse, acoustic refinement member, {cfg.steps} steps (t = 0.3125)",
                     "threads": used, "seconds": el, "mlups": N * N * cfg.steps / el / 1e6,
                     "E_r": O.rms_error(O.phi(p, g), W.pulse_reference(cfg, f))})
    phi_cross = None
    if cross_check:
        cfg = W.PulseConfig(N=1024, steps=1000, D_variable=True)
        rate = allc["value"] * 1e6
        projected = 1024 * 1024 * cfg.steps / max(rate, 1.0)
        entry = {"workload": "1024^2 rotating pulse, D(x) = 1e-3 (1 + 0.5 sin(pi x) sin(pi y)), 1000 steps "
                             "(the precision study's oracle cross-check)", "threads": threads,
                 "projected_seconds": projected}
        if projected <= cross_budget_s:
            g, p, f, el, used = timed_run(cfg, cfg.steps, threads)
            phi_cross = O.phi(p, g)
            entry.update(seconds=el, mlups=1024 * 1024 * cfg.steps / el / 1e6, threads=used,
                         mass=O.mass(phi_cross))
        else:
            entry["skipped"] = f"projected {projected:.0f} s > {cross_budget_s:.0f} s on this host"
        legs.append(entry)
    out = {"value": allc["value"], "unit": "MLUPS", "cores": allc["threads"], "kind": "oracle",
           "sample": f"{n}^2 rotating pulse (the benchmark workload), {kt} of 3200 steps, FP64 plain C oracle, "
                     f"OpenMP over rows on {allc['threads']} threads, {allc['seconds']:.1f} s",
           "single_thread": {"value": single["value"], "unit": "MLUPS", "cores": 1,
                             "sample": f"{n}^2 rotating pulse, {k1} of 3200 steps, 1 thread, {single['seconds']:.1f} s"},
           "host": host, "workloads": legs}
    return out, phi_cross


def oracle_cross_check(torch, W, lbm, Solver, phi_orc):
    """The GPU storage modes on the precision study's cross-check size (1024^2, 1000 steps, variable
    D) against the FP64 oracle's phi of the same run (computed in the CPU-baseline leg): max and L2
    errors, and E_r against the constant-D closed form (context: D varies)."""
    import numpy as np
    cfg = W.PulseConfig(N=1024, steps=1000, D_variable=True)
    f = W.rotating_pulse(cfg)
    dev = {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy", "D")}
    ref = torch.from_numpy(W.pulse_reference(cfg, f)).cuda()
    orc = torch.from_numpy(np.ascontiguousarray(phi_orc)).cuda()
    out = {"N": 1024, "steps": 1000, "D": "1e-3 (1 + 0.5 sin(pi x) sin(pi y))"}
    for mode in ("f64", "f64s_f32m", "f32", "f16s", "f16sr"):
        s = Solver([(lbm.make_params(1024, 1024, f["dx"], f["dt"], cfg.lam, cfg.D, mode), dev)])
        s.step(cfg.steps)
        st, phi = s.macros(ref=ref, want_phi=True, raise_nonfinite=False)
        s.close()
        d = (phi - orc).abs()
        out[mode] = {"max_err_vs_oracle": float(d.max()),
                     "max_rel_err_vs_oracle": float(d.max() / orc.abs().max()),
                     "l2_rel_err_vs_oracle": float(torch.sqrt((d * d).sum() / (orc * orc).sum())),
                     "E_r_vs_constant_D_closed_form": st["rms_err"], "nonfinite": st["nonfinite"]}
    return out


KERNEL_MODES = {"0": "f64", "1": "f64s_f32m", "2": "f32", "3": "f16s", "4": "f16sr"}
TRACE_STEPS = {2048: 1000, 8192: 100}  # timed steps of the kernel-trace runs
PROFILE_STEPS = {"batched": 200, "adjoint": 400, "flux": 100}  # --steps of the profile workloads


def _csv_rows(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(dirpath, suffix):
    for root, _, files in os.walk(dirpath):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {dirpath}")


def _kernel3_label(name: str):
    """'step3_kernel<27, 2, 0, false, false, 0, false, 0>' (velocities, mode, aux, has_k, has_s, walk, cached
    stores, in-place step) -> ('d3q27', 'f32') for the constant-D, source-free kernels; copy -> ('copy',);
    other -> None."""
    import re
    m = re.search(r"step3_kernel<(19|27), (\d), (\d), false, false(?:, \d)?(?:, (?:true|false))?(?:, \d)?>", name)
    if m:
        return (f"d3q{m.group(1)}", KERNEL_MODES[m.group(2)])
    if "copy_kernel" in name:
        return ("copy",)
    return None


def bytes_per_lup3(q: int, mode: str) -> int:
    """Algorithmic HBM bytes per 3D lattice update: q populations in + q out and u (3 components)."""
    return {"f64": 2 * q * 8 + 24, "f64s_f32m": 2 * q * 8 + 12, "f32": 2 * q * 4 + 12, "f16s": 2 * q * 2 + 12}[mode]


def run_profile3(torch, W, lbm, Solver, n, steps):
    """The workload the 3D profiles are taken on: the rotating pulse at n^3 on D3Q19 and D3Q27, FP32,
    FP64 and FP16S storage, `steps` steps each in the default launch shape, then the copy calibration."""
    import numpy as np
    cfg = W.PulseConfig(N=n, steps=steps)
    f = W.rotating_pulse3(cfg)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    fields = {"phi0": dv(f["phi0"]), "ux": dv(f["u"][0]), "uy": dv(f["u"][1]), "uz": dv(f["u"][2])}
    out = {}
    for q in (19, 27):
        for mode in ("f32", "f64", "f16s"):
            s = Solver([(lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode, nz=n, lattice=q), fields)])
            s.step(2)  # graph capture happens outside the timed steps
            ms = _timed_steps(torch, s, steps)
            s.close()
            out[f"d3q{q}_{mode}"] = {"mlups": n ** 3 / (ms * 1e-3) / 1e6, "ms_per_step": ms}
            print(f"# d3q{q} {mode}: {out[f'd3q{q}_{mode}']['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    out["copy_gbps"] = copy_bandwidth(torch, lbm)
    return out


# Profiles of the other hot kernels: the batched step (256 instances), the adjoint (512^2 x 400 steps,
# checkpointed) and the one-step flux form (2048^2 or 8192^2).  Each workload runs its kernels, then
# the copy calibration; summarize_workload() reads one kernel-trace run and one FETCH_SIZE and one
# WRITE_SIZE run of it.
PROFILE_WORKLOADS = ("batched", "adjoint", "flux")


def run_profile_workload(torch, W, lbm, Solver, name, n, steps):
    import numpy as np
    out = {"workload": name}
    if name == "batched":
        draws = W.batched_instances(256, steps=steps)
        insts = []
        for d in draws:
            cfg = d.config
            f = W.rotating_pulse(cfg)
            p = lbm.make_params(cfg.N, cfg.N, f["dx"], f["dt"], cfg.lam, cfg.D, "f32")
            insts.append((p, {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy")}))
        s = Solver(insts)
        nodes = int(sum(d.N * d.N for d in draws))
        for label in ("two_steps_per_launch", "one_step_per_launch"):  # the default, then one step per launch
            if label == "one_step_per_launch":
                s.set_launch(1, 1, tile_width=64)
            s.step(64)
            ms = _timed_steps(torch, s, steps)
            out[label] = {"mlups": nodes / (ms * 1e-3) / 1e6, "launch": s.get_launch()}
        out.update(nodes=nodes, batch=s.get_batch())
        s.close()
    elif name == "adjoint":
        out.update(run_adjoint(torch, W, lbm, Solver))
    elif name == "flux":
        cfg = W.PulseConfig(N=n, steps=steps)
        f = W.rotating_pulse(cfg)
        dev = {k: torch.from_numpy(f[k]).cuda() for k in ("phi0", "ux", "uy")}
        for mode in ("f32", "f64"):
            s = Solver([(lbm.make_params(n, n, f["dx"], f["dt"], cfg.lam, cfg.D, mode, lbm.LBM_AUX_FLUX), dev)])
            for label in ("two_steps_per_launch", "one_step_per_launch"):  # the default, then one step
                if label == "one_step_per_launch":
                    s.set_launch(2, 1, tile_width=256)
                s.step(64)
                ms = _timed_steps(torch, s, steps)
                out[f"{mode}_{label}"] = {"mlups": n * n / (ms * 1e-3) / 1e6, "launch": s.get_launch()}
            s.close()
        del dev
        torch.cuda.empty_cache()
    else:
        raise ValueError(f"unknown profile workload {name}")
    out["copy_gbps"] = copy_bandwidth(torch, lbm)
    return out


def _workload_kernels(name: str, n: int):
    """(label, regex on the kernel name, algorithmic bytes per launch, lattice updates per launch) of
    the kernels a profile workload is about."""
    if name == "batched":
        import workloads as W
        nodes = sum(d.N * d.N for d in W.batched_instances(256))
        return [("batched_step2_kernel FP32, 256 instances, two steps per launch", r"batched_step2_kernel<2, 0, \d>",
                 nodes * 80.0, 2 * nodes),
                ("batched_step_kernel FP32, 256 instances, one step per launch", r"batched_step_kernel<2, 0, \d>",
                 nodes * 80.0, nodes)]
    if name == "adjoint":
        import workloads as W
        nodes = W.C5_N ** 2
        # state 9 x 4 B and lam 9 x 4 B in, lam 9 x 4 B out, u 8 B and k 4 B in, dL/dD (FP64) read and written
        return [("adjoint_kernel FP32 (D field, local aux)", r"adjoint_kernel<2, true, false, true>", nodes * 136.0, nodes),
                ("step_kernel FP32, D field (recomputation, one step per launch)", r"step_kernel<2, 0, true, false, 0, false",
                 nodes * 84.0, nodes),
                ("step2_kernel FP32, D field (forward, two steps per launch)", r"step2_kernel<2, 0, true, false", nodes * 84.0,
                 2 * nodes)]
    if name == "flux":
        return [("flux2_kernel FP32, two steps per launch", r"flux2_kernel<2, false, false", float(n) * n * 80.0, 2 * n * n),
                ("flux2_kernel FP64, two steps per launch", r"flux2_kernel<0, false, false", float(n) * n * 160.0,
                 2 * n * n),
                ("step_kernel FP32, flux form, one step per launch", r"step_kernel<2, 1, false, false", float(n) * n * 80.0,
                 n * n),
                ("step_kernel FP64, flux form, one step per launch", r"step_kernel<0, 1, false, false", float(n) * n * 160.0,
                 n * n)]
    raise ValueError(name)


def summarize_workload(name, n, trace_dir, pmc_dirs, out_dir, command, pmc_commands):
    """profiles/<name>_kernel_profile[_n].md: per kernel of the workload the trace's calls and average
    duration, MLUPS and algorithmic GB/s from it, and the copy-calibrated FETCH_SIZE + WRITE_SIZE bytes
    per launch against the algorithmic bytes."""
    import re
    kernels = _workload_kernels(name, n)
    stats = _csv_rows(_find(trace_dir, "kernel_stats.csv"))
    per, calib = {}, {}
    for counter, d in pmc_dirs.items():
        vals, cal = {}, []
        for r in _csv_rows(_find(d, "counter_collection.csv")):
            if r.get("Counter_Name") != counter:
                continue
            kn = r.get("Kernel_Name", "")
            if "copy_kernel" in kn and "cached" not in kn:
                cal.append(float(r["Counter_Value"]))
            for lab, rx, _, _ in kernels:
                if re.search(rx, kn):
                    vals.setdefault(lab, []).append(float(r["Counter_Value"]))
        if cal:
            calib[counter] = sorted(cal)[len(cal) // 2] / (2 * 1024 * 1024)  # copy moves 2 GiB each way
        for lab, v in vals.items():
            v = sorted(v)
            per.setdefault(lab, {})[counter] = v[len(v) // 2]
    size = f" at {n}^2" if name == "flux" else ""
    md = [f"# rocprofv3 profile: {name} workload{size}", "",
          f"Kernel sources hash: {kernel_hash()}.", "", f"- trace: `{command}`"] + [f"- counters: `{c}`" for c in pmc_commands] + [
          "", "FETCH_SIZE and WRITE_SIZE (KiB per dispatch, median) are divided by what they read for the library's "
              "2 GiB copy kernel in the same run.", "",
          "| kernel | calls | average (us) | MLUPS | algorithmic GB/s | of 8 TB/s | FETCH KiB | WRITE KiB | "
          "counted bytes/launch | algorithmic bytes/launch | ratio |", "|---|---|---|---|---|---|---|---|---|---|---|"]
    for lab, rx, alg, lups in kernels:
        rows = [r for r in stats if re.search(rx, r["Name"])]
        if not rows:
            continue
        calls = sum(int(r["Calls"]) for r in rows)
        total = sum(float(r["TotalDurationNs"]) for r in rows)
        avg = total / calls
        gbps = alg / (avg * 1e-9) / 1e9
        c = per.get(lab, {})
        fetch, write = c.get("FETCH_SIZE"), c.get("WRITE_SIZE")
        if fetch is not None and write is not None and "FETCH_SIZE" in calib and "WRITE_SIZE" in calib:
            hbm = 1024.0 * (fetch / calib["FETCH_SIZE"] + write / calib["WRITE_SIZE"])
            cnt = f"{fetch:.0f} | {write:.0f} | {hbm:.4g} | {alg:.4g} | {hbm / alg:.3f}"
        else:
            cnt = f" | | | {alg:.4g} | "
        md.append(f"| {lab} | {calls} | {avg / 1e3:.2f} | {lups / (avg * 1e-9) / 1e6:.0f} | {gbps:.0f} | "
                  f"{gbps / HBM_PEAK_GBPS:.3f} | {cnt} |")
    fn = f"{name}_kernel_profile" + (f"_{n}" if name == "flux" else "") + ".md"
    with open(os.path.join(out_dir, fn), "w") as fh:
        fh.write("\n".join(md) + "\n")


def summarize_profiles3(trace_dir, pmc_dirs, out_dir, n, command, pmc_commands):
    """Kernel-trace statistics and copy-scaled FETCH_SIZE / WRITE_SIZE traffic of the D3Q19 and D3Q27
    step kernels (written beside the two-dimensional summaries)."""
    lines = [f"# rocprofv3 kernel trace: D3Q19 / D3Q27 step kernels, rotating pulse {n}^3", "",
             f"Command: `{command}`", "",
             "| kernel | lattice | mode | calls | average (us) | total (ms) |", "|---|---|---|---|---|---|"]
    for r in _csv_rows(_find(trace_dir, "kernel_stats.csv")):
        lab = _kernel3_label(r["Name"])
        if lab is None or lab[0] == "copy":
            continue
        lines.append(f"| {r['Name'][:80]} | {lab[0]} | {lab[1]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} |")
    with open(os.path.join(out_dir, f"step3_kernel_trace_{n}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    entries, calib = {}, {}
    for counter, d in pmc_dirs.items():
        per = {}
        for r in _csv_rows(_find(d, "counter_collection.csv")):
            lab = _kernel3_label(r.get("Kernel_Name", ""))
            if lab is None or r.get("Counter_Name") != counter:
                continue
            per.setdefault("copy" if lab[0] == "copy" else f"{lab[0]}_{lab[1]}", []).append(float(r["Counter_Value"]))
        if "copy" in per:
            c = sorted(per.pop("copy"))
            calib[counter] = c[len(c) // 2] / (2 * 1024 * 1024)  # copy moves 2 GiB each way
        for key, vals in per.items():
            vals = sorted(vals)
            entries.setdefault(key, {})[counter + "_KiB_median"] = vals[len(vals) // 2]
    md = [f"# HBM traffic of the D3Q19 / D3Q27 step kernels at {n}^3 (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
          "Each counter is divided by what it reads for the library's 2 GiB copy kernel in the same run. "
          f"Kernel sources hash: {kernel_hash()}.", ""] + [
          f"- `{c}`" for c in pmc_commands] + [
          "", "| lattice | mode | FETCH KiB/dispatch | WRITE KiB/dispatch | HBM bytes/launch | algorithmic bytes/launch | "
              "ratio |", "|---|---|---|---|---|---|---|"]
    for key in sorted(entries):
        e = entries[key]
        lat, mode = key.split("_", 1)
        if "FETCH_SIZE_KiB_median" not in e or "WRITE_SIZE_KiB_median" not in e:
            continue
        hbm = 1024.0 * (e["FETCH_SIZE_KiB_median"] / calib.get("FETCH_SIZE", 1.0) +
                        e["WRITE_SIZE_KiB_median"] / calib.get("WRITE_SIZE", 1.0))
        alg = float(n) ** 3 * bytes_per_lup3(int(lat[3:]), mode)
        e.update(bytes_per_launch=hbm, algorithmic_bytes_per_launch=alg, traffic_over_algorithmic=hbm / alg)
        md.append(f"| {lat} | {mode} | {e['FETCH_SIZE_KiB_median']:.0f} | {e['WRITE_SIZE_KiB_median']:.0f} | "
                  f"{hbm:.4g} | {alg:.4g} | {hbm / alg:.3f} |")
    with open(os.path.join(out_dir, f"step3_kernel_traffic_{n}.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    return entries


def _kernel_label(name: str):
    """'step_kernel<2, 0, false, false, 0, false, 1, false, 0>' (mode, aux, has_k, has_s, boundary, MRT-R,
    walk, cached stores, in-place step) -> ('step', 'f32', aux 0, has_k, has_s) for the periodic TRT-R
    kernels, any store kind or in-place step; copy -> ('copy',); other -> None."""
    import re
    m = re.search(r"step_kernel<(\d), (\d), (true|false), (true|false), 0, false, \d(?:, (?:true|false))?(?:, \d)?>",
                  name)
    if m:
        return ("step", KERNEL_MODES[m.group(1)], int(m.group(2)), m.group(3) == "true", m.group(4) == "true")
    # two steps per launch: step2_kernel<mode, aux, has_k, has_s, MRT, interior waves, cached stores>
    m = re.search(r"step2_kernel<(\d), (\d), (true|false), (true|false), false, \d, (?:true|false)>", name)
    if m:
        return ("step2", KERNEL_MODES[m.group(1)], int(m.group(2)), m.group(3) == "true", m.group(4) == "true")
    if "copy_kernel" in name:
        return ("copy",)
    return None


def summarize_trace(trace_dir, out_dir, n, command):
    """Kernel-trace statistics of the D2Q9 step kernels of one run (profiles/step_kernel_trace_<n>.md),
    with each mode's MLUPS and algorithmic GB/s recomputed from the average kernel duration."""
    os.makedirs(out_dir, exist_ok=True)
    lines = [f"# rocprofv3 kernel trace: TRT-R D2Q9 step kernels, rotating pulse {n}^2 (constant D)", "",
             f"Command: `{command}`", "",
             "| kernel | mode | calls | average (us) | total (ms) | MLUPS | algorithmic GB/s | of 8 TB/s |",
             "|---|---|---|---|---|---|---|---|"]
    stats = _csv_rows(_find(trace_dir, "kernel_stats.csv"))
    per_mode = {}

    def rates(mode, avg_ns, steps=1):
        """MLUPS and algorithmic GB/s of a launch of `steps` steps over the n^2 lattice (a fused launch
        moves the state and fields once for two updates of every node)."""
        if mode == "-":
            return "", "", ""
        mlups = steps * float(n) * n / (avg_ns * 1e-9) / 1e6
        gbps = float(n) * n * bytes_per_lup(mode, False) / (avg_ns * 1e-9) / 1e9
        return f"{mlups:.0f}", f"{gbps:.0f}", f"{gbps / HBM_PEAK_GBPS:.3f}"

    for r in stats:
        lab = _kernel_label(r["Name"])
        if lab is None:
            continue
        mode = lab[1] if lab[0] in ("step", "step2") else "-"
        steps = 2 if lab[0] == "step2" else 1
        avg = float(r["AverageNs"])
        lines.append(f"| {r['Name'][:80]} | {mode} | {r['Calls']} | {avg / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | " + " | ".join(rates(mode, avg, steps)) + " |")
        if mode != "-" and steps == 1:
            per_mode.setdefault(mode, []).append((int(r["Calls"]), float(r["TotalDurationNs"])))
    for mode, ks in sorted(per_mode.items()):
        if len(ks) > 1:  # a one-buffer instance alternates two kernels: their launches together
            calls, total = sum(k[0] for k in ks), sum(k[1] for k in ks)
            lines.append(f"| all step kernels of the mode (alternating in-place steps) | {mode} | {calls} | "
                         f"{total / calls / 1e3:.2f} | {total / 1e6:.2f} | " + " | ".join(rates(mode, total / calls)) + " |")
    with open(os.path.join(out_dir, f"step_kernel_trace_{n}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_profiles(trace_dirs, pmc_dirs, out_dir, commands, pmc_commands):
    """Writes the committed text summaries of rocprofv3 runs: kernel-trace statistics per lattice size
    (trace_dirs, commands: {n: ...}) and the FETCH_SIZE / WRITE_SIZE traffic per dispatch, scaled by
    the copy kernel's reading."""
    os.makedirs(out_dir, exist_ok=True)
    for n, d in trace_dirs.items():
        summarize_trace(d, out_dir, n, commands[n])

    entries, calib = {}, {}
    for (counter, n), d in pmc_dirs.items():
        rows = _csv_rows(_find(d, "counter_collection.csv"))
        per = {}
        for r in rows:
            lab = _kernel_label(r.get("Kernel_Name", ""))
            if lab is None or r.get("Counter_Name") != counter:
                continue
            key = "copy" if lab[0] == "copy" else lab[1]
            per.setdefault(key, []).append(float(r["Counter_Value"]))
        copy_kib = sorted(per.pop("copy"))[len(per.get("copy", [])) // 2] if "copy" in per else None
        if copy_kib is not None:
            calib[(counter, n)] = copy_kib / (2 * 1024 * 1024)  # copy moves 2 GiB each way
        for mode, vals in per.items():
            used = vals[2:] if len(vals) > 4 else vals  # dispatch order; the first two meet cold caches
            e = entries.setdefault(f"{mode}_{n}", {})
            e[counter + "_KiB_mean"] = sum(used) / len(used)  # a mean: in-place steps alternate two kernels
            e[counter + "_dispatches"] = len(used)
    for key, e in entries.items():
        mode, n = key.rsplit("_", 1)
        n = int(n)
        fac_f = calib.get(("FETCH_SIZE", n), 1.0)
        fac_w = calib.get(("WRITE_SIZE", n), 1.0)
        e["fetch_scale"], e["write_scale"] = fac_f, fac_w
        if "FETCH_SIZE_KiB_mean" in e and "WRITE_SIZE_KiB_mean" in e:
            e["bytes_per_launch"] = 1024.0 * (e["FETCH_SIZE_KiB_mean"] / fac_f + e["WRITE_SIZE_KiB_mean"] / fac_w)
            e["algorithmic_bytes_per_launch"] = float(n) * n * bytes_per_lup(mode, False)
            e["traffic_over_algorithmic"] = e["bytes_per_launch"] / e["algorithmic_bytes_per_launch"]
    out = {"kernel_hash": kernel_hash(), "commands": pmc_commands, "entries": entries,
           "copy_scale": {f"{c}_{n}": v for (c, n), v in calib.items()}}
    with open(os.path.join(out_dir, "step_kernel_pmc.json"), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    md = ["# HBM traffic of the step kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE, one counter per run)", "",
          "Each counter is divided by what it reads for the library's 2 GiB copy kernel (scale = KiB read / "
          "KiB moved).", ""] + [f"- `{c}`" for c in pmc_commands] + [
          "", "| mode | N | FETCH KiB/dispatch | WRITE KiB/dispatch | fetch scale | write scale | HBM bytes/launch | "
              "algorithmic bytes/launch | ratio |", "|---|---|---|---|---|---|---|---|---|"]
    for key in sorted(entries):
        e = entries[key]
        mode, n = key.rsplit("_", 1)
        md.append(f"| {mode} | {n} | {e.get('FETCH_SIZE_KiB_mean', float('nan')):.0f} | "
                  f"{e.get('WRITE_SIZE_KiB_mean', float('nan')):.0f} | {e['fetch_scale']:.3f} | {e['write_scale']:.3f} | "
                  f"{e.get('bytes_per_launch', float('nan')):.4g} | {e.get('algorithmic_bytes_per_launch', float('nan')):.4g} | "
                  f"{e.get('traffic_over_algorithmic', float('nan')):.3f} |")
    with open(os.path.join(out_dir, "step_kernel_traffic.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--modes", default="f32,f64,f64s_f32m,f16s,f16sr")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the 8192^2 precision, refinement, flux-form and adjoint studies")
    ap.add_argument("--summarize", metavar="RUNDIR",
                    help="write profiles/ summaries from rocprofv3 output under RUNDIR (no GPU needed)")
    ap.add_argument("--profile3d", type=int, metavar="N", default=0,
                    help="run only the D3Q19/D3Q27 profile workload at N^3 (--steps steps per kernel)")
    ap.add_argument("--profile", choices=PROFILE_WORKLOADS,
                    help="run only one profile workload (batched, adjoint, or the flux form at --n), --steps steps")
    args = ap.parse_args()
    if args.summarize:
        d = args.summarize
        # 256^3 (streaming) under trace3/, pmc3_*; 128^3 (held in the Infinity Cache) under trace3_128/, pmc3_*_128
        for n3, sfx in ((256, ""), (128, "_128")):
            if not os.path.isdir(os.path.join(d, "trace3" + sfx)):
                continue
            pmc3 = {c: os.path.join(d, f"pmc3_{c.lower()}{sfx}") for c in ("FETCH_SIZE", "WRITE_SIZE")}
            pmc3 = {k: v for k, v in pmc3.items() if os.path.isdir(v)}
            summarize_profiles3(os.path.join(d, "trace3" + sfx), pmc3, os.path.join(ROOT, "profiles"), n3,
                                f"rocprofv3 --kernel-trace --stats --output-format csv -d RUNDIR/trace3{sfx} -o trace -- "
                                f"python3 bench.py --profile3d {n3} --steps 100",
                                [f"rocprofv3 --pmc {c} --output-format csv -d RUNDIR/pmc3_{c.lower()}{sfx} -o pmc -- "
                                 f"python3 bench.py --profile3d {n3} --steps 8" for c in sorted(pmc3)])
        for name in PROFILE_WORKLOADS:
            for n in ((2048, 8192) if name == "flux" else (0,)):
                sfx = f"{name}_{n}" if n else name
                tdir = os.path.join(d, f"trace_{sfx}")
                if not os.path.isdir(tdir):
                    continue
                steps = PROFILE_STEPS[name]
                nflag = f" --n {n}" if n else ""
                pmcw = {c: os.path.join(d, f"pmc_{c.lower()}_{sfx}") for c in ("FETCH_SIZE", "WRITE_SIZE")}
                pmcw = {k: v for k, v in pmcw.items() if os.path.isdir(v)}
                summarize_workload(name, n, tdir, pmcw, os.path.join(ROOT, "profiles"),
                                   f"rocprofv3 --kernel-trace --stats --output-format csv -d RUNDIR/trace_{sfx} -o trace -- "
                                   f"python3 bench.py --profile {name}{nflag} --steps {steps}",
                                   [f"rocprofv3 --pmc {c} --output-format csv -d RUNDIR/pmc_{c.lower()}_{sfx} -o pmc -- "
                                    f"python3 bench.py --profile {name}{nflag} --steps {steps}" for c in sorted(pmcw)])
        traces = {n: os.path.join(d, f"trace_{n}") for n in (2048, 8192)}
        traces = {n: v for n, v in traces.items() if os.path.isdir(v)}
        pmc = {(c, n): os.path.join(d, f"pmc_{c.lower()}_{n}") for c in ("FETCH_SIZE", "WRITE_SIZE") for n in (2048, 8192)}
        pmc = {k: v for k, v in pmc.items() if os.path.isdir(v)}
        if not traces and not pmc:
            return
        summarize_profiles(traces, pmc, os.path.join(ROOT, "profiles"),
                           {n: f"rocprofv3 --kernel-trace --stats --output-format csv -d RUNDIR/trace_{n} -o trace -- "
                               f"python3 bench.py --n {n} --steps {TRACE_STEPS[n]} --warmup 10 --modes f32,f64,f16s,f16sr "
                               f"--no-cpu --no-batched --no-studies" for n in traces},
                           [f"rocprofv3 --pmc {c} --output-format csv -d RUNDIR/pmc_{c.lower()}_{n} -o pmc -- "
                            f"python3 bench.py --n {n} --steps 12 --warmup 0 --modes f32,f64,f16s,f16sr --no-cpu --no-batched --no-studies"
                            for (c, n) in sorted(pmc)])
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2312_10316_amd import Solver, lbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lbm.lib()  # the HIP library is required
    if args.profile3d:
        print(json.dumps(run_profile3(torch, W, lbm, Solver, args.profile3d, args.steps)))
        return
    if args.profile:
        print(json.dumps(run_profile_workload(torch, W, lbm, Solver, args.profile, args.n, args.steps), default=str))
        return

    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    head = "f32" if "f32" in modes else modes[0]
    results, phis = {}, {}
    for m in modes:
        results[m], phis[m] = run_mode(m, args.n, args.steps, args.warmup, torch, W, lbm, Solver)
        print(f"# {m}: {results[m]['mlups']:.0f} MLUPS, {results[m]['ms_per_step']:.4f} ms/step, "
              f"E_r {results[m]['E_r']:.4e}", file=sys.stderr, flush=True)
    if "f64" in phis:
        ref = phis["f64"]
        for m in modes:
            d = (phis[m] - ref).abs()
            results[m]["max_err_vs_f64"] = float(d.max())
            results[m]["l2_err_vs_f64"] = float(torch.sqrt((d * d).sum() / (ref * ref).sum()))
            results[m]["speedup_vs_f64"] = results[m]["mlups"] / results["f64"]["mlups"]
    for m in modes:
        bpl = launch_bytes_per_lup(m, False, results[m]["launch"])
        results[m]["bytes_per_lup"] = bpl
        results[m]["hbm_gbps_algorithmic"] = results[m]["mlups"] * 1e6 * bpl / 1e9
        results[m]["roofline_frac"] = results[m]["hbm_gbps_algorithmic"] / HBM_PEAK_GBPS

    copy_gbps = copy_bandwidth(torch, lbm)
    # two buffers of 92 MiB (184 MiB, the size of the in-place 2048^2 FP32 state) stay in the cache
    cache_copy_gbps = copy_bandwidth(torch, lbm, nbytes=92 << 20, reps=50, cached=True)
    r = results[head]
    n2 = float(args.n) ** 2
    achieved = r["hbm_gbps_algorithmic"]
    traffic = traffic_from_profile(head, args.n)
    stores = r["launch"]["stores"]
    out = {
        "metric": METRIC,
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "f64s_f32m": "f64-store/f32", "f16s": "f16-store/f32",
                  "f16sr": "f16-store (stochastic rounding)/f32"}[head],
        "data": "synthetic",
        "config": {"workload": f"rotating Gaussian pulse, periodic {args.n}^2, c=10, U0=pi, D=1e-3, Lambda=1/4, "
                               f"{args.warmup}+{args.steps} steps", "N": args.n, "storage": head,
                   "aux": "local (Eq. 16)"},
        "roofline": {"bound": roofline_bound(stores),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_unit": "bytes/launch filled into L2 from the fabric (rocprofv3 FETCH_SIZE+WRITE_SIZE, "
                                     "copy-calibrated; HBM plus Infinity Cache hits)",
                     "algorithmic_bytes_per_launch": int(n2 * bytes_per_lup(head, False)),
                     "bytes_per_lup": r["bytes_per_lup"], "lups_per_launch": int(n2 * r["launch"]["fuse"]),
                     "steps_per_launch": r["launch"]["fuse"],
                     "single_step_equivalent_gbps": round(r["mlups"] * bytes_per_lup(head, False) / 1e3, 1),
                     "peak_note": "8 TB/s is the HBM3E spec; a state held in the Infinity Cache is served partly "
                                  "from that cache, whose ceiling is the measured cached copy below",
                     "cache_copy_gbps_measured": round(cache_copy_gbps, 1),
                     "frac_of_cache_copy": round(achieved / cache_copy_gbps, 4),
                     "hbm_copy_gbps_measured": round(copy_gbps, 1),
                     "frac_of_hbm_copy": round(achieved / copy_gbps, 4),
                     "state": {0: "two buffers streamed from HBM (non-temporal stores)",
                               1: "two buffers held in the 256 MiB Infinity Cache (cached stores)",
                               2: "one buffer updated in place, held in the 256 MiB Infinity Cache"}[stores]},
        "modes": {m: {k: (round(v, 6) if isinstance(v, float) and abs(v) >= 1e-3 else v) for k, v in results[m].items()}
                  for m in modes},
    }
    if not args.no_studies:
        t0 = time.perf_counter()
        hbm = run_hbm(torch, W, lbm, Solver)
        h = hbm["f32"]
        fz = h["launch"]["fuse"]
        out["roofline_hbm"] = {"bound": "hbm", "kernel": ("step2_kernel FP32, two steps per launch" if fz == 2 else
                                                          "step_kernel FP32, one row per wave") + ", non-temporal stores",
                               "workload": hbm["workload"], "achieved": round(h["achieved_gbps"], 1),
                               "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(h["frac"], 4),
                               "traffic": h["traffic"],
                               "algorithmic_bytes_per_launch": int(8192 ** 2 * bytes_per_lup("f32", False)),
                               "bytes_per_lup": h["bytes_per_lup"], "lups_per_launch": 8192 ** 2 * fz,
                               "steps_per_launch": fz, "mlups": round(h["mlups"], 1),
                               "hbm_copy_gbps_measured": round(copy_gbps, 1),
                               "frac_of_hbm_copy": round(h["achieved_gbps"] / copy_gbps, 4)}
        out["hbm"] = hbm
        print(f"# hbm: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = run_batched(torch, W, lbm, Solver)
        print(f"# batched: {out['batched']['batched']['mlups']:.0f} MLUPS vs serial graph "
              f"{out['batched']['serial_graph']['mlups']:.0f}, eager {out['batched']['serial_eager']['mlups']:.0f}",
              file=sys.stderr, flush=True)
    if not args.no_studies:
        for name, fn in (("precision_8192_variable_D", run_precision_8192), ("refinement", run_refinement),
                         ("flux_aux", run_flux), ("dirichlet_sec3", run_dirichlet),
                         ("tau2_sweep_walls", run_tau2_sweep), ("d3q19", run_3d),
                         ("d3q27", lambda *a: run_3d(*a, q=27)),
                         ("adjoint_512", run_adjoint)):
            t0 = time.perf_counter()
            try:
                out[name] = fn(torch, W, lbm, Solver)
            except Exception as e:  # a failed study is reported, not fatal to the line
                out[name] = {"error": f"{type(e).__name__}: {e}"}
            print(f"# {name}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if not args.no_cpu:
        t0 = time.perf_counter()
        out["cpu_baseline"], phi_orc = cpu_baseline(args.n, cross_check=not args.no_studies)
        print(f"# cpu_baseline: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        if phi_orc is not None:
            out["oracle_cross_check_1024"] = oracle_cross_check(torch, W, lbm, Solver, phi_orc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
