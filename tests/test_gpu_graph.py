"""pond_step captured in a HIP graph and replayed.

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
