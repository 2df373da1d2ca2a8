"""HIP path vs the CPU oracle, element by element, on seeded synthetic inputs.

Bar: FP64 path within 1e-12 (relative to the field's scale) of the oracle in
fixed-iteration mode; adaptive mode within 1e-9 with matching pass counts away
from the App. E threshold; FP32-mixed path within the per-field tolerances
stated in the tests.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1806_05089_amd import pond, workloads
from tests.parity import rel_err, state_errors

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _cfg(w, q=4, **kw):
    ny, nx = w.shape
    base = dict(nx=nx, ny=ny, q1d=q, isothermal=w.isothermal, bc_x=w.bc_x, bc_y=w.bc_y,
                tau=w.tau)
    base.update(kw)
    return pond.PondConfig(**base)


def _ocfg(c: pond.PondConfig):
    return oracle.OracleConfig(q=c.q1d, isothermal=c.isothermal, bc_x=c.bc_x, bc_y=c.bc_y,
                               max_iter=c.max_iter, fixed_iter=c.fixed_iter,
                               seed_mode=c.seed_mode, tau=c.tau, eps_abs=c.eps_abs,
                               eps_rel=c.eps_rel)


def _run_both(w, cfg, nsteps=1):
    """Same initial fields through both sides; returns (gpu f,g,iters), (oracle f,g,iters)."""
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    out, _ = pond.step(cfg, st, nsteps=nsteps)
    torch.cuda.synchronize()
    f0, g0 = oracle.init(w.rho, w.ux, w.uy, w.T, q=cfg.q1d)
    oc = _ocfg(cfg)
    for _ in range(nsteps):
        f0, g0, it, stt = oracle.step(f0, g0, oc)
    gpu = (out.f.double().cpu().numpy(), out.g.cpu().numpy(), out.iters.cpu().numpy())
    return gpu, (f0, g0, it, stt)


def _u_scale(w):
    return max(1e-3, float(np.max(np.hypot(w.ux, w.uy))))


CASES_FIXED = [
    # name, workload factory, q, fixed passes
    ("smooth_thermal_48x40", lambda: workloads.random_smooth(48, 40, seed=1), 4, 3),
    ("tgv32_isothermal", lambda: workloads.taylor_green(32), 4, 2),
    ("sod_96x3_zero_gradient", lambda: workloads.sod(96, 3), 4, 3),
    ("mach5_24x20", lambda: workloads.mach5(24, seed=0), 4, 2),
    ("ragged_67x5", lambda: workloads.random_smooth(67, 5, seed=2, mach=0.6), 4, 3),
    ("d2q9_smooth_40x36", lambda: workloads.random_smooth(40, 36, seed=3, T0=1.0 / 3.0, mach=0.2), 3, 3),
    # T = 50: each node's stencils span ~37 columns, more than a wave walks
    # jointly, and reach past the LDS window (HBM collocation points)
    ("hot_gas_48x40", lambda: workloads.random_smooth(48, 40, seed=12, T0=50.0, dT=0.1, mach=0.3),
     4, 2),
]


@pytest.mark.parametrize("name,make,q,npass", CASES_FIXED, ids=[c[0] for c in CASES_FIXED])
def test_step_fp64_fixed_iter(gpu, name, make, q, npass):
    print(f"case {name}", flush=True)
    w = make()
    cfg = _cfg(w, q=q, fixed_iter=npass)
    (fg, gg, ig), (fo, go, io, so) = _run_both(w, cfg)
    errs = state_errors(fg, gg, fo, go, u_scale=_u_scale(w), T_scale=float(np.max(w.T)))
    assert max(errs.values()) < TOL64, errs
    assert np.all((ig & pond.POND_ITERS_MASK) == npass)


CASES_ADAPTIVE = [
    ("smooth_thermal_48x40", lambda: workloads.random_smooth(48, 40, seed=4), 4),
    ("tgv32_isothermal", lambda: workloads.taylor_green(32), 4),
    ("sod_128x2", lambda: workloads.sod(128, 2), 4),
    ("d2q9_smooth", lambda: workloads.random_smooth(40, 36, seed=5, T0=1.0 / 3.0, mach=0.2), 3),
    # sharp quadrant interfaces: nodes needing 6..20 passes finish in the
    # block's 16-lane tail
    ("riemann2d_64", lambda: workloads.riemann2d(64, seed=3), 4),
]


@pytest.mark.parametrize("name,make,q", CASES_ADAPTIVE, ids=[c[0] for c in CASES_ADAPTIVE])
def test_step_fp64_adaptive(gpu, name, make, q):
    print(f"case {name}", flush=True)
    w = make()
    cfg = _cfg(w, q=q, max_iter=20)
    (fg, gg, ig), (fo, go, io, so) = _run_both(w, cfg)
    same = (ig & pond.POND_ITERS_MASK) == io
    assert same.mean() > 0.98, same.mean()
    errs = state_errors(fg, gg, fo, go, u_scale=_u_scale(w), T_scale=float(np.max(w.T)))
    # nodes that stopped one pass apart differ by about the App. E tolerance
    assert max(errs.values()) < 1e-9, errs
    if same.all():
        assert max(errs.values()) < TOL64, errs


def test_adaptive_tail_runs_and_counts(gpu):
    """The Riemann interfaces need up to max_iter passes at t = 0: the step
    statistics must count them as the oracle does."""
    w = workloads.riemann2d(64, seed=3)
    cfg = _cfg(w, max_iter=20)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    out, stats = pond.step(cfg, st, stats=True)
    f0, g0 = oracle.init(w.rho, w.ux, w.uy, w.T, q=4)
    _, _, io, _ = oracle.step(f0, g0, _ocfg(cfg))
    ig = out.iters.cpu().numpy()
    assert stats["max_iters"] == int(np.max(io & pond.POND_ITERS_MASK)) == 20
    assert np.sum(ig & pond.POND_ITERS_MASK > 8) > 100
    assert stats["nonconverged"] == int(np.sum((ig & pond.POND_ITERS_NONCONVERGED) != 0))
    assert abs(stats["mean_iters"] - float(np.mean(ig & pond.POND_ITERS_MASK))) < 1e-12


HIST_CASES = [
    ("smooth_thermal_48x40", lambda: workloads.random_smooth(48, 40, seed=4), 4),
    ("riemann2d_64", lambda: workloads.riemann2d(64, seed=3), 4),
    ("d2q9_smooth", lambda: workloads.random_smooth(40, 36, seed=5, T0=1.0 / 3.0, mach=0.2), 3),
]


@pytest.mark.parametrize("name,make,q", HIST_CASES, ids=[c[0] for c in HIST_CASES])
def test_iteration_histogram(gpu, name, make, q):
    """pond_stats.iter_hist (App. E's per-node iteration counts as one
    histogram, reduced on the device) against the step's own pass plane and
    against the oracle's per-node counts: equal bin for bin where every node
    took the oracle's count, and off by at most the nodes that did not."""
    print(f"case {name}", flush=True)
    w = make()
    cfg = _cfg(w, q=q, max_iter=20)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    out, stats = pond.step(cfg, st, stats=True)
    ig = out.iters.cpu().numpy() & pond.POND_ITERS_MASK
    hist = np.array(stats["iter_hist"])
    assert hist.shape == (64,) and hist[0] == 0 and hist.sum() == ig.size
    assert np.array_equal(hist, np.bincount(ig.ravel(), minlength=64))
    assert stats["max_iters"] == int(np.max(np.nonzero(hist)[0]))
    f0, g0 = oracle.init(w.rho, w.ux, w.uy, w.T, q=q)
    _, _, io, _ = oracle.step(f0, g0, _ocfg(cfg))
    ho = np.bincount(io.ravel(), minlength=64)
    ndiff = int(np.sum(io != ig))
    assert np.sum(np.abs(hist - ho)) <= 2 * ndiff, (hist[:12], ho[:12], ndiff)
    if ndiff == 0:
        assert np.array_equal(hist, ho)


@pytest.mark.parametrize("nsteps", [1, 2, 5])
def test_multi_step_pingpong(gpu, nsteps):
    w = workloads.taylor_green(24, mach=0.1)
    cfg = _cfg(w, fixed_iter=2)
    (fg, gg, _), (fo, go, _, _) = _run_both(w, cfg, nsteps=nsteps)
    errs = state_errors(fg, gg, fo, go, u_scale=0.1)
    assert max(errs.values()) < TOL64, errs


def test_init_and_moments(gpu):
    w = workloads.random_smooth(33, 17, seed=7, mach=1.5)
    for q, prec in ((4, pond.POND_F64), (3, pond.POND_F64), (4, pond.POND_F32_MIXED)):
        cfg = _cfg(w, q=q, precision=prec)
        T = w.T if q == 4 else w.T / 3.0
        st = pond.init(cfg, w.rho, w.ux, w.uy, T)
        rho, ux, uy, Tm, M = (a.cpu().numpy() for a in pond.moments(cfg, st, raw=True))
        f0, g0 = oracle.init(w.rho, w.ux, w.uy, T, q=q)
        ro, uxo, uyo, To, Mo = oracle.moments(f0, g0, q=q, with_raw=True)
        tol = 1e-13 if prec == pond.POND_F64 else 2e-7
        assert rel_err(st.f.double().cpu().numpy(), f0) < tol
        assert np.array_equal(st.g.cpu().numpy(), g0)
        assert rel_err(rho, ro) < tol
        assert rel_err(ux, uxo, 1.0) < 10 * tol and rel_err(uy, uyo, 1.0) < 10 * tol
        assert rel_err(Tm, To) < 10 * tol
        assert rel_err(M, Mo) < 10 * tol


CASES_FP32 = [
    ("smooth_thermal_48x40", lambda: workloads.random_smooth(48, 40, seed=8, mach=0.5), 4),
    ("d2q9_smooth_40x36", lambda: workloads.random_smooth(40, 36, seed=9, T0=1.0 / 3.0, mach=0.3), 3),
    ("tgv32_isothermal", lambda: workloads.taylor_green(32, mach=0.2), 4),
    ("sod_96x3_zero_gradient", lambda: workloads.sod(96, 3), 4),
    ("ragged_67x5", lambda: workloads.random_smooth(67, 5, seed=2, mach=0.6), 4),
    ("strip_1x7", lambda: workloads.random_smooth(1, 7, seed=17, mach=0.4), 4),
]


@pytest.mark.parametrize("name,make,q", CASES_FP32, ids=[c[0] for c in CASES_FP32])
def test_fp32_mixed_vs_oracle(gpu, name, make, q):
    """FP32 bulk arithmetic, FP64 transfer rows and convergence test."""
    w = make()
    cfg = _cfg(w, q=q, precision=pond.POND_F32_MIXED, fixed_iter=3)
    (fg, gg, _), (fo, go, _, _) = _run_both(w, cfg)
    # velocities relative to the thermal speed (a field at rest, like the
    # tube's u_y, carries FP32 rounding noise of ~1e-8 sqrt(T))
    u_scale = max(_u_scale(w), float(np.sqrt(np.max(w.T))))
    errs = state_errors(fg, gg, fo, go, u_scale=u_scale, T_scale=float(np.max(w.T)))
    # single-step error of FP32 arithmetic (eps32 = 6e-8) through ~300 terms
    assert errs["f"] < 2e-6 and errs["ux"] < 2e-6 and errs["uy"] < 2e-6 and errs["T"] < 2e-6, errs


def test_edge_single_node_and_strips(gpu):
    for nx, ny in ((1, 1), (1, 7), (9, 1), (2, 2)):
        w = workloads.random_smooth(nx, ny, seed=nx * 10 + ny, mach=0.4)
        cfg = _cfg(w, fixed_iter=2)
        (fg, gg, _), (fo, go, _, _) = _run_both(w, cfg)
        errs = state_errors(fg, gg, fo, go, u_scale=1.0, T_scale=1.0)
        assert max(errs.values()) < TOL64, (nx, ny, errs)


def test_zero_gradient_both_axes(gpu):
    w = workloads.riemann2d(40, seed=3)
    cfg = _cfg(w, fixed_iter=3)
    (fg, gg, _), (fo, go, _, _) = _run_both(w, cfg)
    errs = state_errors(fg, gg, fo, go, u_scale=_u_scale(w), T_scale=float(np.max(w.T)))
    assert max(errs.values()) < TOL64, errs


def test_seed_modes_match_oracle(gpu):
    w = workloads.random_smooth(32, 32, seed=9, mach=0.2)
    for mode in (1, 2):
        cfg = _cfg(w, seed_mode=mode, max_iter=40)
        (fg, gg, ig), (fo, go, io, so) = _run_both(w, cfg)
        errs = state_errors(fg, gg, fo, go, u_scale=_u_scale(w), T_scale=float(np.max(w.T)))
        assert max(errs.values()) < 1e-9, (mode, errs)


def test_stats_and_bad_state(gpu):
    w = workloads.random_smooth(40, 24, seed=11)
    cfg = _cfg(w, max_iter=1)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    out, stats = pond.step(cfg, st, stats=True)
    it = out.iters.cpu().numpy()
    assert stats["max_iters"] == 1 and stats["bad_state"] == 0
    assert stats["nonconverged"] == int(np.count_nonzero(it & pond.POND_ITERS_NONCONVERGED))
    assert stats["nonconverged"] > 0
    # a state with T <= 0 at one node (forced from the host): flagged, NaN output, no error
    g = st.g.clone()
    g[2, 5, 7] = -1.0
    bad_in = pond.PondState(st.f.clone(), g, st.iters.clone())
    cfg2 = _cfg(w, max_iter=20)
    out2, stats2 = pond.step(cfg2, bad_in, stats=True)
    it2 = out2.iters.cpu().numpy()
    assert stats2["bad_state"] == int(np.count_nonzero(it2 & pond.POND_ITERS_BAD)) > 0
    assert np.isnan(out2.g.cpu().numpy()[:, it2 & pond.POND_ITERS_BAD > 0]).all()


def test_init_rejects_bad_fields(gpu):
    w = workloads.uniform(8, 8)
    cfg = _cfg(w)
    T = w.T.copy()
    T[3, 3] = 0.0
    with pytest.raises(pond.PondError) as e:
        pond.init(cfg, w.rho, w.ux, w.uy, T)
    assert e.value.code == -4


def test_full_size_sampled_riemann_1024(gpu):
    """1024^2 four-quadrant Riemann input in the benchmark's launch configuration,
    checked against the oracle at 384 sampled nodes (all quadrants, interfaces, edges)."""
    w = workloads.riemann2d(1024, seed=3)
    rng = np.random.default_rng(0)
    for prec, tol in ((pond.POND_F64, TOL64), (pond.POND_F32_MIXED, 2e-6)):
        cfg = _cfg(w, precision=prec, max_iter=20)
        if prec == pond.POND_F32_MIXED:
            cfg = cfg.replace(eps_abs=1e-6, eps_rel=1e-5, fixed_iter=3)
        else:
            cfg = cfg.replace(fixed_iter=3)
        st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        out, _ = pond.step(cfg, st)
        f_in = st.f.double().cpu().numpy()
        g_in = st.g.cpu().numpy()
        N = 1024
        pts = list(rng.integers(0, N * N, 256))
        for y in (0, 1, 511, 512, 1022, 1023):
            for x in (0, 2, 510, 511, 512, 513, 1023):
                pts.append(y * N + x)
        pts = np.array(pts[:384], dtype=np.int64)
        fo, go, io, so = oracle.step_nodes(f_in, g_in, _ocfg(cfg), pts)
        fg = out.f.double().cpu().numpy().reshape(16, -1)[:, pts]
        gg = out.g.cpu().numpy().reshape(3, -1)[:, pts]
        errs = state_errors(fg, gg, fo, go, u_scale=1.0, T_scale=float(np.max(w.T)))
        assert max(errs.values()) < tol, (prec, errs)


def test_full_size_sampled_riemann_2048(gpu):
    """The 2048^2 Riemann input (the largest benchmark grid, 8192 tiles): both
    precisions with fixed passes at 320 sampled nodes, tile seams and corners."""
    N = 2048
    w = workloads.riemann2d(N, seed=3)
    rng = np.random.default_rng(7)
    pts = list(rng.integers(0, N * N, 256))
    for y in (0, 15, 16, 1023, 1024, 2047):
        for x in (0, 31, 32, 1023, 1024, 1025, 2016, 2047):
            pts.append(y * N + x)
    pts = np.array(pts, dtype=np.int64)
    for prec, tol in ((pond.POND_F64, TOL64), (pond.POND_F32_MIXED, 2e-6)):
        cfg = _cfg(w, precision=prec, max_iter=20, fixed_iter=3)
        if prec == pond.POND_F32_MIXED:
            cfg = cfg.replace(eps_abs=1e-6, eps_rel=1e-5)
        st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        out, _ = pond.step(cfg, st)
        fo, go, _, _ = oracle.step_nodes(st.f.double().cpu().numpy(), st.g.cpu().numpy(),
                                         _ocfg(cfg), pts)
        fg = out.f.double().cpu().numpy().reshape(16, -1)[:, pts]
        gg = out.g.cpu().numpy().reshape(3, -1)[:, pts]
        errs = state_errors(fg, gg, fo, go, u_scale=1.0, T_scale=float(np.max(w.T)))
        assert max(errs.values()) < tol, (prec, errs)
        del st, out


def test_large_grid_sampled_riemann_4096(gpu):
    """A 4096^2 grid (16.8 M nodes, 32768 tiles, 2.1 GB per FP64 population
    buffer), beyond the benchmark sizes: FP64 with fixed passes at 256 sampled
    nodes including the last rows and columns (index arithmetic past 2^31
    bytes per buffer)."""
    N = 4096
    w = workloads.riemann2d(N, seed=3)
    rng = np.random.default_rng(11)
    pts = list(rng.integers(0, N * N, 224))
    for y in (0, 2047, 4095):
        for x in (0, 31, 2048, 4064, 4095):
            pts.append(y * N + x)
    pts = np.array(pts, dtype=np.int64)
    cfg = _cfg(w, max_iter=20, fixed_iter=3)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    out, stats = pond.step(cfg, st, stats=True)
    assert stats["bad_state"] == 0
    f_in = st.f.cpu().numpy()
    g_in = st.g.cpu().numpy()
    del st
    fo, go, _, _ = oracle.step_nodes(f_in, g_in, _ocfg(cfg), pts)
    fg = out.f.cpu().numpy().reshape(16, -1)[:, pts]
    gg = out.g.cpu().numpy().reshape(3, -1)[:, pts]
    errs = state_errors(fg, gg, fo, go, u_scale=1.0, T_scale=float(np.max(w.T)))
    assert max(errs.values()) < TOL64, errs


def test_full_size_sampled_riemann_1024_adaptive(gpu):
    """The benchmark's own configuration (adaptive passes, 16-lane tail) on the
    1024^2 Riemann input: sampled nodes, including the 64 that take the most
    passes (they finish in the tail), against the oracle.  Pass counts agree at
    almost every node; where they do the states agree to 1e-9."""
    w = workloads.riemann2d(1024, seed=3)
    cfg = _cfg(w, max_iter=20)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    st, _ = pond.step(cfg, st, nsteps=20)
    out, _ = pond.step(cfg, st.clone())
    f_in = st.f.double().cpu().numpy()
    g_in = st.g.cpu().numpy()
    it = out.iters.cpu().numpy().reshape(-1) & pond.POND_ITERS_MASK
    rng = np.random.default_rng(1)
    pts = np.concatenate([np.argsort(it)[-64:], rng.integers(0, it.size, 192)]).astype(np.int64)
    assert it[pts[:64]].max() > 7  # past the bulk-pass cap: finished in the tail
    fo, go, io, _ = oracle.step_nodes(f_in, g_in, _ocfg(cfg), pts)
    same = (io & pond.POND_ITERS_MASK) == it[pts]
    assert np.mean(same) >= 0.95, np.mean(same)
    fg = out.f.double().cpu().numpy().reshape(16, -1)[:, pts]
    gg = out.g.cpu().numpy().reshape(3, -1)[:, pts]
    errs = state_errors(fg[:, same], gg[:, same], fo[:, same], go[:, same], u_scale=1.0,
                        T_scale=float(np.max(w.T)))
    assert max(errs.values()) < 1e-9, errs


def test_full_size_sampled_riemann_1024_d2q9(gpu):
    """The benchmark's D2Q9 line (the Riemann input with temperatures scaled to
    T_L = 1/3, 1024^2): both precisions with fixed passes at 384 sampled nodes,
    then FP64 with adaptive passes after 20 steps at 256 nodes including the
    64 that take the most passes."""
    w = workloads.riemann2d(1024, seed=3, T_scale=workloads.TL_D2Q9)
    N = 1024
    rng = np.random.default_rng(5)
    pts = list(rng.integers(0, N * N, 256))
    for y in (0, 1, 511, 512, 1022, 1023):
        for x in (0, 2, 510, 511, 512, 513, 1023):
            pts.append(y * N + x)
    pts = np.array(pts[:384], dtype=np.int64)
    for prec, tol in ((pond.POND_F64, TOL64), (pond.POND_F32_MIXED, 2e-6)):
        cfg = _cfg(w, q=3, precision=prec, max_iter=20, fixed_iter=3)
        if prec == pond.POND_F32_MIXED:
            cfg = cfg.replace(eps_abs=1e-6, eps_rel=1e-5)
        st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        out, _ = pond.step(cfg, st)
        fo, go, _, _ = oracle.step_nodes(st.f.double().cpu().numpy(), st.g.cpu().numpy(),
                                         _ocfg(cfg), pts)
        fg = out.f.double().cpu().numpy().reshape(9, -1)[:, pts]
        gg = out.g.cpu().numpy().reshape(3, -1)[:, pts]
        errs = state_errors(fg, gg, fo, go, u_scale=1.0, T_scale=float(np.max(w.T)))
        assert max(errs.values()) < tol, (prec, errs)
    cfg = _cfg(w, q=3, max_iter=20)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    st, _ = pond.step(cfg, st, nsteps=20)
    out, _ = pond.step(cfg, st.clone())
    it = out.iters.cpu().numpy().reshape(-1) & pond.POND_ITERS_MASK
    sel = np.concatenate([np.argsort(it)[-64:], rng.integers(0, it.size, 192)]).astype(np.int64)
    fo, go, io, _ = oracle.step_nodes(st.f.double().cpu().numpy(), st.g.cpu().numpy(),
                                      _ocfg(cfg), sel)
    same = (io & pond.POND_ITERS_MASK) == it[sel]
    assert np.mean(same) >= 0.95, np.mean(same)
    fg = out.f.double().cpu().numpy().reshape(9, -1)[:, sel]
    gg = out.g.cpu().numpy().reshape(3, -1)[:, sel]
    errs = state_errors(fg[:, same], gg[:, same], fo[:, same], go[:, same], u_scale=1.0,
                        T_scale=float(np.max(w.T)))
    assert max(errs.values()) < 1e-9, errs


def _far_base(q):
    return workloads.random_smooth(48, 40, seed=13, mach=0.3, T0=1.0 if q == 4 else 1.0 / 3.0)


@pytest.mark.parametrize("q", [4, 3])
def test_far_stencils_fixed_passes(gpu, q):
    """Departure points 300 nodes upstream: such nodes leave the wave's joint
    column walk and finish in the block tail.  Checked against the oracle at
    the same velocities; the oracle's lab-frame moments (eqs. 10-12 as
    printed) cancel terms of size |u|^2, so its own rounding is ~|u|^2 eps."""
    U = 300.0
    w = workloads.shifted(_far_base(q), U)
    cfg = _cfg(w, q=q, fixed_iter=2)
    (fg, gg, ig), (fo, go, io, _) = _run_both(w, cfg)
    tol = 10.0 * U * U * np.finfo(np.float64).eps
    errs = state_errors(fg, gg, fo, go, u_scale=U, T_scale=float(np.max(w.T)))
    assert max(errs.values()) < tol, (tol, errs)
    assert np.all((ig & pond.POND_ITERS_MASK) == 2)


def test_far_stencils_adaptive_galilean(gpu):
    """Converged steps are Galilean invariant under integer shifts, so the
    adaptive run at u + 300 equals the oracle's run at u rolled by 300 nodes
    per step, with 300 added to u_x (to the App. E tolerance).  A truncated
    iteration is not: its seed is the node's own stored gauge, which the
    shift does not move."""
    base = _far_base(4)
    w = workloads.shifted(base, 300.0)
    cfg = _cfg(w, max_iter=20)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    out, _ = pond.step(cfg, st, nsteps=2)
    f0, g0 = oracle.init(base.rho, base.ux, base.uy, base.T, q=4)
    oc = _ocfg(_cfg(base, max_iter=20))
    for _ in range(2):
        f0, g0, io, _ = oracle.step(f0, g0, oc)
    shift = (300 * 2) % 48
    fo, go = np.roll(f0, shift, axis=-1), np.roll(g0, shift, axis=-1)
    go[0] += 300.0
    # (pass counts differ with the seeds; the converged values do not)
    errs = state_errors(out.f.double().cpu().numpy(), out.g.cpu().numpy(), fo, go,
                        u_scale=300.0, T_scale=float(np.max(w.T)))
    assert max(errs.values()) < 1e-9, errs


def test_tile_order_multi_step_ragged(gpu):
    """A multi-tile ragged grid (100 x 90: 4 x 6 tiles of 32 x 16, both edges
    partial) stepped four times in one call and then four more times one call
    at a time: each step takes its tiles in the order the previous step left,
    and every tile must still be computed exactly once."""
    w = workloads.random_smooth(100, 90, seed=11, mach=0.8)
    cfg = _cfg(w, fixed_iter=2)
    (fg, gg, _), (fo, go, _, _) = _run_both(w, cfg, nsteps=4)
    errs = state_errors(fg, gg, fo, go, u_scale=_u_scale(w))
    assert max(errs.values()) < TOL64, errs
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    for _ in range(4):
        st, _ = pond.step(cfg, st)
    assert torch.equal(st.f, torch.from_numpy(fg).to(st.f.device))
    assert torch.equal(st.g, torch.from_numpy(gg).to(st.g.device))


def test_tile_order_precision_switch(gpu):
    """FP32-mixed and FP64 steps use different tile shapes (32 x 8 and 32 x 16):
    alternating them on one stream and grid must not hand one precision the
    tile order the other left (every tile is still computed exactly once, so
    the FP32-mixed run repeats bit for bit)."""
    w = workloads.riemann2d(96, seed=3)
    c32 = _cfg(w, precision=pond.POND_F32_MIXED, max_iter=20, eps_abs=1e-6, eps_rel=1e-5)
    c64 = _cfg(w, max_iter=20)
    runs = []
    for _ in range(2):
        st = pond.init(c32, w.rho, w.ux, w.uy, w.T)
        out, _ = pond.step(c32, st, nsteps=3)
        runs.append((out.f.clone(), out.g.clone(), out.iters.clone()))
        s64 = pond.init(c64, w.rho, w.ux, w.uy, w.T)
        pond.step(c64, s64, nsteps=3)
    for a, b in zip(runs[0], runs[1]):
        assert torch.equal(a, b)
    assert int((runs[0][2] & pond.POND_ITERS_MASK).min()) >= 1


def test_tile_arrays_across_lattices_and_grids(gpu):
    """D2Q16 and D2Q9 steps of both precisions on grids of different tile
    counts, interleaved on one stream (the library's tile arrays grow to the
    largest grid and each step keys and orders only its own tiles): each run
    repeats bit for bit."""
    cases = []
    for n, q in ((96, 4), (160, 3), (64, 4), (200, 3)):
        w = workloads.riemann2d(n, seed=3, T_scale=1.0 if q == 4 else workloads.TL_D2Q9)
        for prec in (pond.POND_F64, pond.POND_F32_MIXED):
            kw = dict(precision=prec, max_iter=20)
            if prec == pond.POND_F32_MIXED:
                kw.update(eps_abs=1e-6, eps_rel=1e-5)
            cases.append((w, _cfg(w, q=q, **kw)))
    runs = [[], []]
    for r in range(2):
        for w, cfg in cases:
            st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
            out, _ = pond.step(cfg, st, nsteps=3)
            runs[r].append((out.f.clone(), out.g.clone(), out.iters.clone()))
    for a, b in zip(runs[0], runs[1]):
        for x, y in zip(a, b):
            assert torch.equal(x, y)


@pytest.mark.parametrize("prec", [pond.POND_F64, pond.POND_F32_MIXED])
def test_results_independent_of_tile_order_1024(gpu, prec):
    """At 1024^2 (over two tiles per block in the queue) a block takes its next
    tile, and in FP64 that tile's seed gauges, while it finishes the current
    one; which tiles go that way depends on the tile order.  The same
    adaptive steps twice on one stream, the second starting from the order
    the first left, agree bit for bit."""
    w = workloads.riemann2d(1024, seed=3)
    kw = dict(precision=prec, max_iter=20)
    if prec == pond.POND_F32_MIXED:
        kw.update(eps_abs=1e-6, eps_rel=1e-5)
    cfg = _cfg(w, **kw)
    outs = []
    for _ in range(2):
        st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        out, _ = pond.step(cfg, st, nsteps=3)
        outs.append((out.f.clone(), out.g.clone(), out.iters.clone()))
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)


def test_adaptive_results_independent_of_tile_order(gpu):
    """The same adaptive run twice on one stream: the second run starts from
    the tile order the first left behind, and must agree bit for bit."""
    w = workloads.riemann2d(128, seed=3)
    cfg = _cfg(w, max_iter=20)
    outs = []
    for _ in range(2):
        st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        out, stats = pond.step(cfg, st, nsteps=6, stats=True)
        outs.append((out.f.clone(), out.g.clone(), out.iters.clone(), stats))
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][2], outs[1][2])
    assert outs[0][3] == outs[1][3]
