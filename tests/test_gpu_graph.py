"""pond_step and pond_step_adjoint captured in a HIP graph and replayed.

The step path records no memset: the tile queue resets itself at kernel end,
step statistics (which synchronise) are not requested, and an even step count
ends in a device-to-device copy.  Each replay, with the program's own eager
steps and synchronisations in between, must equal the eager result bit for
bit (results do not depend on the tile order either slot carries).
"""
import pytest
import torch

from paper_1806_05089_amd import pond, workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nsteps", [1, 2, 3])
def test_step_graph_replays_match_eager(gpu, nsteps):
    w = workloads.riemann2d(128, seed=3)
    cfg = pond.PondConfig(nx=128, ny=128, bc_x=1, bc_y=1, tau=0.55, max_iter=20)
    st0 = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    ref, _ = pond.step(cfg, st0.clone(), nsteps=nsteps)
    torch.cuda.synchronize()

    src, dst = st0.clone(), pond.empty_state(cfg)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        # the first call on a stream allocates its slot: warm up before capture
        for _ in range(2):
            src.f.copy_(st0.f)
            src.g.copy_(st0.g)
            pond.step(cfg, src, dst, nsteps=nsteps)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pond.step(cfg, src, dst, nsteps=nsteps)

    for replay in range(4):
        src.f.copy_(st0.f)
        src.g.copy_(st0.g)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(dst.f, ref.f), replay
        assert torch.equal(dst.g, ref.g), replay
        assert torch.equal(dst.iters, ref.iters), replay
        # eager work of the program between replays
        other, _ = pond.step(cfg, st0.clone(), nsteps=1)
        torch.cuda.synchronize()
        assert torch.isfinite(other.f).all()


@pytest.mark.parametrize("prec", [pond.POND_F64, pond.POND_F32_MIXED])
def test_adjoint_graph_replays_match_eager(gpu, prec):
    """pond_step_adjoint (its recording step, the zero fills and the adjoint
    kernel) captured and replayed.  The adjoint adds with floating-point
    atomics, whose order varies, so replays agree with the eager result to
    rounding, not bit for bit."""
    w = workloads.riemann2d(96, seed=3)
    cfg = pond.PondConfig(nx=96, ny=80, bc_x=1, bc_y=1, tau=0.55, max_iter=20, precision=prec)
    if prec == pond.POND_F32_MIXED:
        cfg = cfg.replace(eps_abs=1e-6, eps_rel=1e-5)
    rho, ux, uy, T = (a[:80, :96].copy() for a in (w.rho, w.ux, w.uy, w.T))
    st = pond.init(cfg, rho, ux, uy, T)
    st, _ = pond.step(cfg, st, nsteps=5)
    out, _ = pond.step(cfg, st.clone())
    gen = torch.Generator(device="cuda").manual_seed(5)
    wf = torch.randn(out.f.shape, dtype=torch.float64, device="cuda", generator=gen)
    wg = torch.randn(out.g.shape, dtype=torch.float64, device="cuda", generator=gen)
    tau_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    ref_f, ref_g = pond.step_adjoint(cfg, st, out, wf, wg, tau_ref)
    torch.cuda.synchronize()

    atau = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):  # allocates the stream's slot and scratch
            pond.step_adjoint(cfg, st, out, wf, wg, atau)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        af, ag = pond.step_adjoint(cfg, st, out, wf, wg, atau)

    def close(a, b):
        return float(torch.max(torch.abs(a - b))) <= 1e-12 * float(torch.max(torch.abs(b)))

    for replay in range(4):
        atau.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert close(af, ref_f) and close(ag, ref_g), replay
        assert abs(float(atau) - float(tau_ref)) <= 1e-12 * abs(float(tau_ref)), replay
        # eager work of the program between replays
        e_f, _ = pond.step_adjoint(cfg, st, out, wf, wg)
        torch.cuda.synchronize()
        assert torch.isfinite(e_f).all()
