"""Differentiable PonD rollouts: torch.autograd over the hand-written adjoint.

``PondRollout.apply(f0, g0, tau, cfg, nsteps, checkpoint_every)`` runs
``nsteps`` pond_step launches and returns the final (f, g).  Its backward pass
replays each segment of ``checkpoint_every`` steps from the saved state at the
segment start with ``pond_step_record`` (so memory holds nsteps / K checkpoints
plus one segment's states and pass histories) and calls
``pond_step_adjoint_recorded`` step by step in reverse.  Gradients flow to the
initial populations and gauge and to tau (nu = T_ref (tau - 1/2) dt, so
dJ/dnu = (dJ/dtau) / T_ref).

``equilibrium_state`` builds the initial state from macroscopic fields with
pond_init and gives the fields their gradients with pond_init_adjoint (the
equilibrium f = rho W_i W_j is linear in rho; its transpose is the W-weighted
sum over populations, computed in the library).  ``kinetic_energy`` takes the
density from pond_moments.
"""
from __future__ import annotations

import torch

from . import pond
from .pond import PondConfig, PondState


class _Equilibrium(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, ux, uy, T, cfg: PondConfig):
        st = pond.init(cfg, rho.detach(), ux.detach(), uy.detach(), T.detach(), device=rho.device)
        ctx.cfg = cfg
        return st.f, st.g

    @staticmethod
    def backward(ctx, gf, gg):
        cfg = ctx.cfg
        af = gf.double().contiguous() if gf is not None else None
        ag = gg.double().contiguous() if gg is not None else None
        if af is None:
            af = torch.zeros((cfg.Q, cfg.ny, cfg.nx), dtype=torch.float64, device=ag.device)
        if ag is None:
            ag = torch.zeros((3, cfg.ny, cfg.nx), dtype=torch.float64, device=af.device)
        grho, gux, guy, gT = pond.init_adjoint(cfg, af, ag)
        return grho, gux, guy, gT, None


def equilibrium_state(cfg: PondConfig, rho, ux, uy, T):
    """(f, g) = pond_init(rho, u, T), differentiable in the four fields."""
    return _Equilibrium.apply(rho, ux, uy, T, cfg)


class PondRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, g0, tau, cfg: PondConfig, nsteps: int, checkpoint_every: int):
        cfg_t = cfg.replace(tau=float(tau))
        a = PondState(f0.detach().contiguous().clone(), g0.detach().contiguous().clone(),
                      torch.zeros((cfg.ny, cfg.nx), dtype=torch.uint8, device=f0.device))
        b = pond.empty_state(cfg_t, f0.device)
        checkpoints = []
        for k in range(nsteps):
            if k % checkpoint_every == 0:
                checkpoints.append((k, a.f.clone(), a.g.clone()))
            pond.step(cfg_t, a, b)
            a, b = b, a
        ctx.cfg = cfg_t
        ctx.nsteps = nsteps
        ctx.K = checkpoint_every
        ctx.checkpoints = checkpoints
        return a.f.clone(), a.g.clone()

    @staticmethod
    def backward(ctx, gf, gg):
        cfg = ctx.cfg
        dev = ctx.checkpoints[0][1].device
        af = (gf if gf is not None else torch.zeros_like(ctx.checkpoints[0][1])).double().contiguous()
        ag = (gg if gg is not None else torch.zeros_like(ctx.checkpoints[0][2])).double().contiguous()
        atau = torch.zeros(1, dtype=torch.float64, device=dev)
        for k0, f_ck, g_ck in reversed(ctx.checkpoints):
            k1 = min(k0 + ctx.K, ctx.nsteps)
            # replay the segment, keeping every state and the pass history each
            # step records, then run the recorded steps' adjoints backwards
            states = [PondState(f_ck.clone(), g_ck.clone(),
                                torch.zeros((cfg.ny, cfg.nx), dtype=torch.uint8, device=dev))]
            tapes = []
            for _ in range(k0, k1):
                out, tape = pond.step_record(cfg, states[-1])
                states.append(out)
                tapes.append(tape)
            for k in range(k1 - k0, 0, -1):
                af, ag = pond.step_adjoint_recorded(cfg, states[k - 1], states[k], tapes.pop(),
                                                    af, ag, atau)
        return af.to(ctx.checkpoints[0][1].dtype) if cfg.precision == pond.POND_F32_MIXED else af, \
            ag, atau.reshape(()), None, None, None


def rollout(f0, g0, tau, cfg: PondConfig, nsteps: int, checkpoint_every: int = 20):
    """Differentiable nsteps-step rollout; ``tau`` is a 0-d float64 tensor."""
    return PondRollout.apply(f0, g0, tau, cfg, nsteps, checkpoint_every)


class _Density(torch.autograd.Function):
    """rho = sum_p f_p (eq. (10)) from pond_moments; its transpose hands the
    cotangent of rho to every population unchanged."""

    @staticmethod
    def forward(ctx, f, g):
        Q, ny, nx = f.shape
        cfg = PondConfig(nx=nx, ny=ny, q1d=4 if Q == 16 else 3,
                         precision=pond.POND_F64 if f.dtype == torch.float64 else pond.POND_F32_MIXED)
        st = PondState(f.detach().contiguous(), g.detach().contiguous(), None)
        ctx.shape = f.shape
        ctx.dtype = f.dtype
        return pond.moments(cfg, st)[0]

    @staticmethod
    def backward(ctx, grho):
        return grho.to(ctx.dtype).expand(ctx.shape).contiguous(), None


def density(f, g):
    """rho of a state (pond_moments), differentiable in f."""
    return _Density.apply(f, g)


def kinetic_energy(f, g):
    """J = sum over nodes of rho |u|^2 / 2 with rho = sum_p f_p and u the node gauge."""
    rho = density(f, g)
    return 0.5 * (rho * (g[0] * g[0] + g[1] * g[1])).sum()
