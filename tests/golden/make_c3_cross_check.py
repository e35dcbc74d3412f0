"""Writes ``c3_cross_check_1024.json``: the FP64 oracle's result for the cross-check size of the
variable-D precision study, to compare the GPU storage modes against without re-running the oracle.

Workload: rotating Gaussian pulse on the periodic 1024^2 lattice over [-1, 1]^2 (c = dx/dt = 10,
U0 = pi, sigma0 = 0.1 centred at (0.5, 0), Lambda = 1/4), D(x) = 1e-3 (1 + 0.5 sin(pi x) sin(pi y)),
1000 steps of the TRT-R step with the auxiliary term of Eq. (16), no source.  Every value stored here
comes from ``oracle/`` (its OpenMP build, bitwise the single-threaded one) and from the input
module's fields; nothing comes from the HIP library.

Stored: phi at every node of a 32 x 32 window with stride 2 around the pulse maximum and on a
stride-64 grid over the whole lattice; all nine pre-collision populations at an 8 x 8 subset of the
window; the correctly rounded sum of phi over each row; mass; max |phi|; E_r (Eq. (33)) against the
constant-D closed form with D = 1e-3 (context only: D varies).

    python tests/golden/make_c3_cross_check.py [--threads 0]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c3_cross_check_1024.json")
N, STEPS = 1024, 1000


def window(phi):
    """Origin (row, column) of the stride-2 32 x 32 window centred on the maximum of phi."""
    k, j = np.unravel_index(int(np.argmax(phi)), phi.shape)
    return int(k) - 32, int(j) - 32


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    cfg = W.PulseConfig(N=N, steps=STEPS, D_variable=True)
    f = W.rotating_pulse(cfg)
    p = O.Problem(N, N, f["dx"], f["dt"], cfg.lam, cfg.D, O.AUX_LOCAL)
    g0 = O.init(p, f["phi0"], f["ux"], f["uy"])
    t0 = time.perf_counter()
    g, threads = O.run_threads(p, g0, STEPS, f["ux"], f["uy"], D=f["D"], threads=args.threads)
    el = time.perf_counter() - t0
    phi = O.phi(p, g)
    k0, j0 = window(phi)
    wk = [(k0 + 2 * a) % N for a in range(32)]
    wj = [(j0 + 2 * b) % N for b in range(32)]
    ck = list(range(0, N, 64))
    pk = wk[::4]
    pj = wj[::4]
    out = {
        "what": "FP64 oracle, rotating pulse 1024^2 periodic on [-1,1]^2, c=10, U0=pi, sigma0=0.1 at (0.5,0), "
                "Lambda=1/4, D(x)=1e-3(1+0.5 sin(pi x) sin(pi y)), 1000 steps, auxiliary term of Eq. (16), no source",
        "written_by": "python tests/golden/make_c3_cross_check.py (calls oracle/ and workloads/ only)",
        "N": N, "steps": STEPS, "t_end": cfg.t_end,
        "oracle_seconds": el, "oracle_threads": threads,
        "window_rows": wk, "window_cols": wj,
        "phi_window": [[float(phi[k, j]) for j in wj] for k in wk],
        "coarse_rows": ck, "coarse_cols": ck,
        "phi_coarse": [[float(phi[k, j]) for j in ck] for k in ck],
        "pop_rows": pk, "pop_cols": pj,
        "pops": [[[float(g[i, k, j]) for j in pj] for k in pk] for i in range(9)],
        "row_sums": [math.fsum(phi[k].tolist()) for k in range(N)],
        "mass": O.mass(phi),
        "max_abs_phi": float(np.abs(phi).max()),
        "E_r_vs_constant_D_closed_form": O.rms_error(phi, W.pulse_reference(cfg, f)),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
        fh.write("\n")
    print(f"wrote {OUT}: oracle {el:.1f} s on {threads} threads, mass {out['mass']:.17g}")


if __name__ == "__main__":
    main()
