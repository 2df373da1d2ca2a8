"""Write sod_rounding_sensitivity.json: how far the oracle's own FP64
trajectory of the 1024 x 4 shock tube (fixed 3 passes, 400 steps) moves when
every step's output is perturbed by one unit of FP64 rounding.

Two oracle runs from the same initial state; in the second, after every step
each population and gauge value is multiplied by (1 + 2^-53 xi), xi uniform in
[-1, 1] (numpy default_rng(0)).  The per-field spread between the runs
(max|a - b| / max(max|b|, scale), scales 1 for f, sqrt(0.25) for u, max T0
for T) at the recorded steps measures the trajectory's amplification of
rounding: any FP64 implementation of the step whose rounding differs from the
oracle's drifts from it by about this spread times its own per-step rounding
difference in units of 2^-53.  Calls only the oracle.

    python tests/golden/make_sod_sensitivity.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1806_05089_amd import workloads  # noqa: E402

STEPS = (1, 10, 40, 100, 200, 300, 400)


def spread(a, b, scale):
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), scale))


def main():
    w = workloads.sod(1024, 4)
    cfg = oracle.OracleConfig(bc_x=1, tau=w.tau, fixed_iter=3)
    f, g = oracle.init(w.rho, w.ux, w.uy, w.T)
    fp, gp = f.copy(), g.copy()
    rng = np.random.default_rng(0)
    u = 2.0 ** -53
    nodes = np.arange(f.shape[1] * f.shape[2])
    u_scale, T_scale = float(np.sqrt(w.meta["scale"])), float(np.max(w.T))
    out = {}
    for n in range(1, STEPS[-1] + 1):
        fs, gs, _, _ = oracle.step_nodes(f, g, cfg, nodes)
        f, g = fs.reshape(f.shape), gs.reshape(g.shape)
        fs, gs, _, _ = oracle.step_nodes(fp, gp, cfg, nodes)
        fp = fs.reshape(f.shape) * (1.0 + u * rng.uniform(-1.0, 1.0, f.shape))
        gp = gs.reshape(g.shape) * (1.0 + u * rng.uniform(-1.0, 1.0, g.shape))
        if n in STEPS:
            out[str(n)] = {"f": spread(fp, f, 1.0), "ux": spread(gp[0], g[0], u_scale),
                           "uy": spread(gp[1], g[1], u_scale), "T": spread(gp[2], g[2], T_scale)}
            print(n, out[str(n)], flush=True)
    rec = {"workload": "sod 1024x4, tau 0.52, zero-gradient x, fixed 3 passes",
           "noise": "each step's output times (1 + 2^-53 xi), xi ~ U[-1, 1], default_rng(0)",
           "unit_noise": u, "spread_by_step": out}
    with open(os.path.join(HERE, "sod_rounding_sensitivity.json"), "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
