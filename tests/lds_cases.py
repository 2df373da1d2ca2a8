"""Cases of the LDS-poison comparison (tests/test_gpu_lds_poison.py).

Run as a script with the library to use in POND_LIBRARY; writes the outputs
of every case to the .npz file named on the command line.  Each case covers a
way into the LDS windows: ragged grids (partial tiles and windows), both
precisions and lattices, zero-gradient edges, the adaptive 16-lane tail,
departure points far outside the window, and the adjoint's staged window.
"""
import sys

import numpy as np
import torch

from paper_1806_05089_amd import pond, workloads


def _case(w, q=4, **kw):
    ny, nx = w.shape
    cfg = pond.PondConfig(nx=nx, ny=ny, q1d=q, isothermal=w.isothermal, bc_x=w.bc_x,
                          bc_y=w.bc_y, tau=w.tau, **kw)
    T = w.T if q == 4 else w.T / 3.0
    st = pond.init(cfg, w.rho, w.ux, w.uy, T)
    return cfg, st


def run():
    out = {}

    def forward(name, w, q=4, nsteps=2, **kw):
        cfg, st = _case(w, q, **kw)
        st, _ = pond.step(cfg, st, nsteps=nsteps)
        torch.cuda.synchronize()
        out[name + "_f"] = st.f.double().cpu().numpy()
        out[name + "_g"] = st.g.cpu().numpy()
        out[name + "_it"] = st.iters.cpu().numpy()

    forward("ragged_f64", workloads.random_smooth(67, 45, seed=31, mach=0.6), fixed_iter=3)
    forward("ragged_f32", workloads.random_smooth(67, 45, seed=31, mach=0.6), fixed_iter=3,
            precision=pond.POND_F32_MIXED)
    forward("d2q9", workloads.random_smooth(53, 37, seed=32, mach=0.3, T0=1.0), q=3,
            fixed_iter=3)
    forward("riemann_adaptive", workloads.riemann2d(96, seed=3), max_iter=20)
    forward("riemann_adaptive_f32", workloads.riemann2d(96, seed=3), max_iter=20,
            precision=pond.POND_F32_MIXED, eps_abs=1e-6, eps_rel=1e-5)
    forward("far_u300", workloads.shifted(workloads.random_smooth(40, 24, seed=33, mach=0.2),
                                          300.0), fixed_iter=2)
    # adjoint (its staged window)
    cfg, st = _case(workloads.random_smooth(48, 40, seed=34, mach=0.4), fixed_iter=3)
    nxt, _ = pond.step(cfg, st)
    rng = np.random.default_rng(35)
    wf = torch.from_numpy(rng.standard_normal(nxt.f.shape)).cuda()
    wg = torch.from_numpy(rng.standard_normal(nxt.g.shape)).cuda()
    af, ag = pond.step_adjoint(cfg, st, nxt, wf, wg)
    torch.cuda.synchronize()
    out["adjoint_f"] = af.cpu().numpy()
    out["adjoint_g"] = ag.cpu().numpy()
    return out


if __name__ == "__main__":
    np.savez(sys.argv[1], **run())
