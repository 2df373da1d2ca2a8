"""Adjoint of pond_step vs the oracle's complex-step derivatives.

The oracle is evaluated in complex arithmetic (complex step, h = 1e-30), which
gives exact directional derivatives of its computed map.  With the pass count
fixed (fixed-iteration mode) the GPU adjoint differentiates the same map, so
  <J delta, w>  (oracle, complex step)  ==  <delta, J^T w>  (GPU adjoint)
to round-off, for random directions delta and cotangents w, and element by
element on a tiny grid.  POND_ADJOINT_LANES selects the one-lane or the
two- or four-lane adjoint kernel (read at every call).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1806_05089_amd import autograd, pond, workloads

pytestmark = pytest.mark.gpu

H = 1e-30


def _ocfg(c: pond.PondConfig):
    return oracle.OracleConfig(q=c.q1d, isothermal=c.isothermal, bc_x=c.bc_x, bc_y=c.bc_y,
                               max_iter=c.max_iter, fixed_iter=c.fixed_iter,
                               seed_mode=c.seed_mode, tau=c.tau, eps_abs=c.eps_abs,
                               eps_rel=c.eps_rel)


def _setup(w, q=4, **kw):
    ny, nx = w.shape
    cfg = pond.PondConfig(nx=nx, ny=ny, q1d=q, isothermal=w.isothermal, bc_x=w.bc_x,
                          bc_y=w.bc_y, tau=w.tau, **kw)
    T = w.T if q == 4 else w.T / 3.0
    st = pond.init(cfg, w.rho, w.ux, w.uy, T)
    # move off equilibrium so every population carries information
    rng = np.random.default_rng(5)
    f = st.f.double().cpu().numpy() * (1.0 + 0.05 * rng.standard_normal(st.f.shape))
    st.f.copy_(torch.from_numpy(f).to(st.f.dtype))
    out, _ = pond.step(cfg, st)
    return cfg, st, out


def _vjp(cfg, st, out, wf, wg):
    atau = torch.zeros(1, dtype=torch.float64, device=st.f.device)
    af, ag = pond.step_adjoint(cfg, st, out, torch.from_numpy(wf).cuda(),
                               torch.from_numpy(wg).cuda(), atau)
    torch.cuda.synchronize()
    return af.cpu().numpy(), ag.cpu().numpy(), float(atau.item())


def _jvp(cfg, f, g, df, dg, dtau=0.0):
    fo, go, _, _ = oracle.step_cs(f + 1j * H * df, g + 1j * H * dg, _ocfg(cfg),
                                  tau=cfg.tau + 1j * H * dtau)
    return fo.imag / H, go.imag / H


CASES = [
    ("thermal_periodic", lambda: workloads.random_smooth(20, 18, seed=1, mach=0.4), 4, {}),
    ("isothermal_tgv", lambda: workloads.taylor_green(16, mach=0.2), 4, {}),
    ("zero_gradient_riemann", lambda: workloads.riemann2d(24, seed=3), 4, {}),
    ("seed_mode_2", lambda: workloads.random_smooth(16, 16, seed=2, mach=0.2), 4, {"seed_mode": 2}),
    ("d2q9", lambda: workloads.random_smooth(18, 16, seed=3, mach=0.2, T0=1.0), 3, {}),
    ("mach5", lambda: workloads.mach5(16, seed=0), 4, {}),
    # departure points 300 nodes upstream: lanes walk their own stencils
    ("far_stencils_u300", lambda: workloads.shifted(workloads.random_smooth(16, 16, seed=6,
                                                                           mach=0.2), 300.0),
     4, {}),
]


@pytest.mark.parametrize("lanes", [1, 2, 4])
@pytest.mark.parametrize("name,make,q,kw", CASES, ids=[c[0] for c in CASES])
def test_dot_product_against_complex_step(gpu, monkeypatch, name, make, q, kw, lanes):
    """Every adjoint kernel: one lane per node (large grids) and two or four
    lanes per node, each taking a share of the y speeds (smaller grids; D2Q16
    only)."""
    if q == 3 and lanes > 1:
        pytest.skip("D2Q9's three y speeds do not split over several lanes")
    monkeypatch.setenv("POND_ADJOINT_LANES", str(lanes))
    print(f"case {name} lanes {lanes}", flush=True)
    w = make()
    cfg, st, out = _setup(w, q=q, fixed_iter=3, **kw)
    f = st.f.double().cpu().numpy()
    g = st.g.cpu().numpy()
    rng = np.random.default_rng(11)
    for trial in range(2):
        df = rng.standard_normal(f.shape) * 1e-2
        dg = rng.standard_normal(g.shape) * np.array([0.1, 0.1, 0.05])[:, None, None]
        if cfg.isothermal:
            dg[2] = 0.0 if trial == 0 else dg[2]
        wf = rng.standard_normal(f.shape)
        wg = rng.standard_normal(g.shape)
        af, ag, atau = _vjp(cfg, st, out, wf, wg)
        jf, jg = _jvp(cfg, f, g, df, dg)
        lhs = float(np.sum(jf * wf) + np.sum(jg * wg))
        rhs = float(np.sum(df * af) + np.sum(dg * ag))
        assert abs(lhs - rhs) <= 1e-9 * max(abs(lhs), 1e-12), (trial, lhs, rhs)
    # d/dtau
    jf, jg = _jvp(cfg, f, g, np.zeros_like(f), np.zeros_like(g), dtau=1.0)
    lhs = float(np.sum(jf * wf) + np.sum(jg * wg))
    assert abs(lhs - atau) <= 1e-9 * max(abs(lhs), 1e-12), (lhs, atau)


def test_vjp_elementwise_tiny_grid(gpu):
    w = workloads.random_smooth(6, 5, seed=4, mach=0.3)
    cfg, st, out = _setup(w, fixed_iter=2)
    f = st.f.double().cpu().numpy()
    g = st.g.cpu().numpy()
    rng = np.random.default_rng(12)
    wf = rng.standard_normal(f.shape)
    wg = rng.standard_normal(g.shape)
    af, ag, _ = _vjp(cfg, st, out, wf, wg)
    ref_f = np.zeros_like(f)
    ref_g = np.zeros_like(g)
    for idx in np.ndindex(*f.shape):
        df = np.zeros_like(f)
        df[idx] = 1.0
        jf, jg = _jvp(cfg, f, g, df, np.zeros_like(g))
        ref_f[idx] = np.sum(jf * wf) + np.sum(jg * wg)
    for idx in np.ndindex(*g.shape):
        dg = np.zeros_like(g)
        dg[idx] = 1.0
        jf, jg = _jvp(cfg, f, g, np.zeros_like(f), dg)
        ref_g[idx] = np.sum(jf * wf) + np.sum(jg * wg)
    assert np.max(np.abs(af - ref_f)) <= 1e-10 * np.max(np.abs(ref_f))
    assert np.max(np.abs(ag - ref_g)) <= 1e-10 * np.max(np.abs(ref_g))


def test_adaptive_mode_dot_product(gpu):
    """Adaptive passes: the adjoint uses the forward's recorded counts; the oracle's
    counts agree at almost every node, so the dot products agree closely."""
    w = workloads.random_smooth(20, 20, seed=6, mach=0.3)
    cfg, st, out = _setup(w, max_iter=20)
    f = st.f.double().cpu().numpy()
    g = st.g.cpu().numpy()
    _, _, it, _ = oracle.step(f, g, _ocfg(cfg))
    assert np.array_equal(it, out.iters.cpu().numpy() & pond.POND_ITERS_MASK)
    rng = np.random.default_rng(13)
    df = rng.standard_normal(f.shape) * 1e-2
    dg = rng.standard_normal(g.shape) * 1e-2
    wf = rng.standard_normal(f.shape)
    wg = rng.standard_normal(g.shape)
    af, ag, _ = _vjp(cfg, st, out, wf, wg)
    jf, jg = _jvp(cfg, f, g, df, dg)
    lhs = float(np.sum(jf * wf) + np.sum(jg * wg))
    rhs = float(np.sum(df * af) + np.sum(dg * ag))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_rollout_gradient_vs_complex_step(gpu):
    """Gradient of the final kinetic energy of a 12-step rollout (checkpoints every 5)
    w.r.t. the initial velocity field and tau, against the oracle's complex step."""
    w = workloads.compressible_taylor_green(16, seed=1)
    ny, nx = w.shape
    cfg = pond.PondConfig(nx=nx, ny=ny, tau=0.6, fixed_iter=3)
    nsteps = 12
    rho = torch.tensor(w.rho, dtype=torch.float64, device="cuda")
    ux = torch.tensor(w.ux, dtype=torch.float64, device="cuda", requires_grad=True)
    uy = torch.tensor(w.uy, dtype=torch.float64, device="cuda", requires_grad=True)
    T = torch.tensor(w.T, dtype=torch.float64, device="cuda")
    tau = torch.tensor(0.6, dtype=torch.float64, device="cuda", requires_grad=True)
    f0, g0 = autograd.equilibrium_state(cfg, rho, ux, uy, T)
    fT, gT = autograd.rollout(f0, g0, tau, cfg, nsteps, checkpoint_every=5)
    J = autograd.kinetic_energy(fT, gT)
    J.backward()
    gux = ux.grad.cpu().numpy()
    gtau = float(tau.grad.item())

    def J_cs(dux, dtau):
        f, g = oracle.init_cs(w.rho, w.ux + 1j * H * dux, w.uy, w.T)
        for _ in range(nsteps):
            f, g, _, _ = oracle.step_cs(f, g, oracle.OracleConfig(tau=0.6, fixed_iter=3),
                                        tau=0.6 + 1j * H * dtau)
        rho_ = f.sum(0)
        return (0.5 * rho_ * (g[0] ** 2 + g[1] ** 2)).sum().imag / H

    rng = np.random.default_rng(2)
    d = rng.standard_normal(w.ux.shape)
    lhs = J_cs(d, 0.0)
    rhs = float(np.sum(gux * d))
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs), (lhs, rhs)
    assert abs(J_cs(np.zeros_like(d), 1.0) - gtau) <= 1e-8 * abs(gtau)
    # and central finite differences (h = 1e-4) on the GPU forward
    h = 1e-4

    def J_gpu(ux_np, tau_v):
        c = cfg.replace(tau=tau_v)
        st = pond.init(c, w.rho, ux_np, w.uy, w.T)
        out, _ = pond.step(c, st, nsteps=nsteps)
        return float(autograd.kinetic_energy(out.f, out.g).item())

    fd = (J_gpu(w.ux + h * d, 0.6) - J_gpu(w.ux - h * d, 0.6)) / (2 * h)
    assert abs(fd - rhs) <= 1e-6 * abs(rhs), (fd, rhs)


@pytest.mark.parametrize("prec", [pond.POND_F64, pond.POND_F32_MIXED])
def test_recorded_step_and_adjoint(gpu, prec):
    """pond_step_record is pond_step bit for bit, and the adjoint about the
    recorded step equals pond_step_adjoint (which records the step itself) to
    rounding (both add with floating-point atomics)."""
    w = workloads.riemann2d(48, seed=3)
    cfg = pond.PondConfig(nx=48, ny=48, bc_x=1, bc_y=1, tau=0.55, max_iter=20, precision=prec)
    if prec == pond.POND_F32_MIXED:
        cfg = cfg.replace(eps_abs=1e-6, eps_rel=1e-5)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    st, _ = pond.step(cfg, st, nsteps=4)
    ref, _ = pond.step(cfg, st.clone())
    rec, tape = pond.step_record(cfg, st.clone())
    assert tape.numel() == pond.tape_bytes(cfg)
    assert torch.equal(rec.f, ref.f) and torch.equal(rec.g, ref.g)
    assert torch.equal(rec.iters, ref.iters)
    gen = torch.Generator(device="cuda").manual_seed(9)
    wf = torch.randn(ref.f.shape, dtype=torch.float64, device="cuda", generator=gen)
    wg = torch.randn(ref.g.shape, dtype=torch.float64, device="cuda", generator=gen)
    t1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    t2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    f1, g1 = pond.step_adjoint(cfg, st, ref, wf, wg, t1)
    f2, g2 = pond.step_adjoint_recorded(cfg, st, rec, tape, wf, wg, t2)
    for a, b in ((f2, f1), (g2, g1)):
        assert float(torch.max(torch.abs(a - b))) <= 1e-12 * float(torch.max(torch.abs(b)))
    assert abs(float(t2) - float(t1)) <= 1e-12 * abs(float(t1))


def test_adjoint_on_caller_workspace(gpu):
    """pond_step_adjoint keeps its scratch in the caller's workspace: one
    filled with garbage and passed at an offset inside a larger buffer gives
    the adjoint of a freshly allocated one to rounding (the adjoint adds with
    floating-point atomics); one byte short is refused before any launch."""
    w = workloads.riemann2d(40, seed=3)
    cfg = pond.PondConfig(nx=40, ny=40, bc_x=1, bc_y=1, tau=0.55, max_iter=20)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    st, _ = pond.step(cfg, st, nsteps=3)
    out, _ = pond.step(cfg, st.clone())
    gen = torch.Generator(device="cuda").manual_seed(4)
    wf = torch.randn(out.f.shape, dtype=torch.float64, device="cuda", generator=gen)
    wg = torch.randn(out.g.shape, dtype=torch.float64, device="cuda", generator=gen)
    nb = pond.workspace_bytes(cfg)
    assert nb >= pond.tape_bytes(cfg)
    big = torch.full((nb + 512,), 0xFF, dtype=torch.uint8, device="cuda")
    t1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    t2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    f1, g1 = pond.step_adjoint(cfg, st, out, wf, wg, t1, workspace=big[256:256 + nb])
    f2, g2 = pond.step_adjoint(cfg, st, out, wf, wg, t2)
    for a, b in ((f1, f2), (g1, g2)):
        assert float(torch.max(torch.abs(a - b))) <= 1e-12 * float(torch.max(torch.abs(b)))
    assert abs(float(t1) - float(t2)) <= 1e-12 * abs(float(t2))
    with pytest.raises(pond.PondError):
        pond.step_adjoint(cfg, st, out, wf, wg, t1, workspace=big[:nb - 1])


@pytest.mark.parametrize("q", [4, 3])
def test_init_adjoint_is_the_transpose_of_init(gpu, q):
    """pond_init_adjoint against pond_init itself: f = rho W is linear in rho,
    so <init(rho), a_f> = <rho, adj_rho> for any rho; the gauge cotangents
    pass through unchanged; adj_rho = sum_p W_p a_f,p with the oracle's
    weights."""
    cfg = pond.PondConfig(nx=13, ny=7, q1d=q)
    rng = np.random.default_rng(q)
    rho = rng.uniform(0.5, 1.5, (7, 13))
    zero = np.zeros((7, 13))
    af = torch.from_numpy(rng.standard_normal((q * q, 7, 13))).cuda()
    ag = torch.from_numpy(rng.standard_normal((3, 7, 13))).cuda()
    ar, aux, auy, aT = (t.cpu().numpy() for t in pond.init_adjoint(cfg, af, ag))
    st = pond.init(cfg, rho, zero, zero, np.ones((7, 13)))
    lhs = float(torch.sum(st.f * af))
    assert abs(lhs - float(np.sum(rho * ar))) <= 1e-13 * abs(lhs)
    agn = ag.cpu().numpy()
    assert np.array_equal(aux, agn[0]) and np.array_equal(auy, agn[1])
    assert np.array_equal(aT, agn[2])
    _, wts, _ = oracle.lattice(q)
    W = np.outer(wts, wts).reshape(-1)
    ref = np.tensordot(W, af.cpu().numpy(), axes=1)
    assert np.max(np.abs(ar - ref)) <= 1e-15 * np.max(np.abs(ref)) * q * q


def test_adjoint_scatter_order_only_moves_rounding(gpu, monkeypatch):
    """The adjoint adds collocation cotangents with floating-point atomics, so
    its result depends on the order in which tiles and lanes add.  Repeated
    calls, and the one-, two- and four-lane kernels (different tiles, a node's
    y speeds split over lanes), must agree to the rounding of those sums:
    1e-13 of the largest entry.  Every element is checked against the
    oracle's complex step by test_vjp_elementwise_tiny_grid; the dot products
    above check multi-tile grids."""
    w = workloads.riemann2d(56, seed=3)
    cfg = pond.PondConfig(nx=56, ny=56, bc_x=1, bc_y=1, tau=0.55, fixed_iter=3)
    st = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    st, _ = pond.step(cfg, st, nsteps=3)
    out, _ = pond.step(cfg, st.clone())
    gen = torch.Generator(device="cuda").manual_seed(7)
    wf = torch.randn(out.f.shape, dtype=torch.float64, device="cuda", generator=gen)
    wg = torch.randn(out.g.shape, dtype=torch.float64, device="cuda", generator=gen)
    runs = []
    for lanes in (1, 1, 1, 2, 4):
        monkeypatch.setenv("POND_ADJOINT_LANES", str(lanes))
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        af, ag = pond.step_adjoint(cfg, st, out, wf, wg, t)
        torch.cuda.synchronize()
        runs.append((lanes, af.cpu().numpy(), ag.cpu().numpy(), float(t.item())))
    _, f0, g0, t0 = runs[0]
    for lanes, f, g, t in runs[1:]:
        ef = np.max(np.abs(f - f0)) / np.max(np.abs(f0))
        eg = np.max(np.abs(g - g0)) / np.max(np.abs(g0))
        print(f"lanes {lanes}: f {ef:.1e} g {eg:.1e} tau {abs(t - t0) / abs(t0):.1e}", flush=True)
        assert ef < 1e-13 and eg < 1e-13 and abs(t - t0) <= 1e-13 * abs(t0)
