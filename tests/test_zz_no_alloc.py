"""pond_step_noalloc (the entry point that allocates nothing) against pond_step.

Both run the same kernels; the no-allocation variant keeps its counters, tile
queue and tile arrays in the library's fixed device array.  Results do not
depend on the tile order, so the two agree bit for bit: on two calls in a row
(the second on a smaller grid, so the array holds the first call's contents),
with statistics and with several steps per call.
"""
import ctypes as C

import pytest
import torch

from paper_1806_05089_amd import _lib, pond, workloads

pytestmark = pytest.mark.gpu


def _cfg(w, **kw):
    ny, nx = w.shape
    return pond.PondConfig(nx=nx, ny=ny, isothermal=w.isothermal, bc_x=w.bc_x, bc_y=w.bc_y,
                           tau=w.tau, max_iter=20, **kw)


def _noalloc_abi(cfg, a, b, nsteps, stats):
    """The call through the C ABI itself (ctypes), no Python wrapper."""
    lib = _lib.load()
    st = _lib.pond_stats()
    ca, cb = a.c(), b.c()
    rc = lib.pond_step_noalloc(C.byref(cfg.c()), C.byref(ca), C.byref(cb), int(nsteps),
                               torch.cuda.current_stream().cuda_stream,
                               C.byref(st) if stats else None)
    assert rc == _lib.POND_OK, lib.pond_last_error()
    return st


@pytest.mark.parametrize("q", [4, 3])
@pytest.mark.parametrize("prec", [pond.POND_F64, pond.POND_F32_MIXED])
def test_noalloc_matches_step_two_calls_second_smaller(gpu, prec, q):
    kw = dict(precision=prec, q1d=q)
    if prec == pond.POND_F32_MIXED:
        kw.update(eps_abs=1e-6, eps_rel=1e-5)
    for n, nsteps in ((200, 3), (72, 2)):
        print(f"case noalloc q {q} prec {prec} grid {n} nsteps {nsteps}", flush=True)
        w = workloads.riemann2d(n, seed=3, T_scale=1.0 if q == 4 else 1.0 / 3.0)
        cfg = _cfg(w, **kw)
        ref_in = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        ref, ref_stats = pond.step(cfg, ref_in, nsteps=nsteps, stats=True)
        a = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        b = pond.empty_state(cfg)
        st = _noalloc_abi(cfg, a, b, nsteps, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(b.f, ref.f) and torch.equal(b.g, ref.g)
        assert torch.equal(b.iters, ref.iters)
        assert st.nonconverged == ref_stats["nonconverged"]
        assert st.bad_state == ref_stats["bad_state"] == 0
        assert st.max_iters == ref_stats["max_iters"]
        assert list(st.iter_hist) == ref_stats["iter_hist"]
        assert sum(st.iter_hist) == n * n


def test_noalloc_repeated_calls_reuse_tile_order(gpu):
    """Steps one call at a time on one grid (the tile order left by one call
    feeds the next) equal one pond_step call of as many steps."""
    w = workloads.riemann2d(160, seed=3)
    cfg = _cfg(w)
    ref, _ = pond.step(cfg, pond.init(cfg, w.rho, w.ux, w.uy, w.T), nsteps=4)
    a = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    b = pond.empty_state(cfg)
    for _ in range(4):
        _noalloc_abi(cfg, a, b, 1, stats=False)
        a, b = b, a
    torch.cuda.synchronize()
    assert torch.equal(a.f, ref.f) and torch.equal(a.g, ref.g)
