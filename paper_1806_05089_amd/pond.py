"""Python face of libpond: the same four calls, taking torch device tensors.

Every step of the method runs in the HIP kernels behind the C ABI; this module
only allocates device tensors, passes their pointers and the current HIP stream,
and raises on a nonzero return code.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _lib
from ._lib import (POND_F32_MIXED, POND_F64, POND_ITERS_BAD, POND_ITERS_MASK,  # noqa: F401
                   POND_ITERS_NONCONVERGED, POND_OP_STEP, POND_OP_STEP_ADJOINT, POND_PERIODIC,
                   POND_ZERO_GRADIENT, PondError)


@dataclasses.dataclass
class PondConfig:
    nx: int
    ny: int
    q1d: int = 4
    precision: int = POND_F64
    isothermal: int = 0
    bc_x: int = POND_PERIODIC
    bc_y: int = POND_PERIODIC
    max_iter: int = 20
    fixed_iter: int = 0
    seed_mode: int = 0
    tau: float = 0.6
    eps_abs: float = 1e-12
    eps_rel: float = 1e-10

    def c(self) -> _lib.pond_config:
        return _lib.pond_config(self.nx, self.ny, self.q1d, self.precision, self.isothermal,
                                self.bc_x, self.bc_y, self.max_iter, self.fixed_iter,
                                self.seed_mode, float(self.tau), float(self.eps_abs),
                                float(self.eps_rel))

    @property
    def Q(self) -> int:
        return self.q1d * self.q1d

    @property
    def fdtype(self) -> torch.dtype:
        return torch.float64 if self.precision == POND_F64 else torch.float32

    def replace(self, **kw) -> "PondConfig":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class PondState:
    f: torch.Tensor      # [Q, ny, nx] float64 or float32
    g: torch.Tensor      # [3, ny, nx] float64
    iters: torch.Tensor  # [ny, nx] uint8

    def c(self) -> _lib.pond_state:
        return _lib.pond_state(self.f.data_ptr(), self.g.data_ptr(),
                               self.iters.data_ptr() if self.iters is not None else None)

    def clone(self) -> "PondState":
        return PondState(self.f.clone(), self.g.clone(), self.iters.clone())


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require(t: torch.Tensor, shape, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)}")


def empty_state(cfg: PondConfig, device="cuda") -> PondState:
    return PondState(torch.empty((cfg.Q, cfg.ny, cfg.nx), dtype=cfg.fdtype, device=device),
                     torch.empty((3, cfg.ny, cfg.nx), dtype=torch.float64, device=device),
                     torch.zeros((cfg.ny, cfg.nx), dtype=torch.uint8, device=device))


def _check_state(cfg: PondConfig, st: PondState, name: str):
    _require(st.f, (cfg.Q, cfg.ny, cfg.nx), cfg.fdtype, name + ".f")
    _require(st.g, (3, cfg.ny, cfg.nx), torch.float64, name + ".g")
    if st.iters is not None:
        _require(st.iters, (cfg.ny, cfg.nx), torch.uint8, name + ".iters")


def init(cfg: PondConfig, rho, ux, uy, T, device="cuda") -> PondState:
    """pond_init: equilibrium state f = rho W in the gauge {u, T}."""
    lib = _lib.load()
    fields = [torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
              for a in (rho, ux, uy, T)]
    for a, n in zip(fields, ("rho", "ux", "uy", "T")):
        _require(a, (cfg.ny, cfg.nx), torch.float64, n)
    st = empty_state(cfg, device)
    cs = st.c()
    _lib.check(lib.pond_init(C.byref(cfg.c()), *[a.data_ptr() for a in fields], C.byref(cs),
                             _stream_ptr(st.f.device)))
    return st


def step(cfg: PondConfig, state_in: PondState, state_out: PondState | None = None,
         nsteps: int = 1, stats: bool = False):
    """pond_step.  Returns (state_out, stats_dict or None).

    With nsteps > 1 the library ping-pongs between the two states, so
    state_in's buffers are overwritten.  stats["iter_hist"][n] counts the
    nodes that took n predictor-corrector passes in the last step."""
    lib = _lib.load()
    _check_state(cfg, state_in, "state_in")
    if state_out is None:
        state_out = empty_state(cfg, state_in.f.device)
    _check_state(cfg, state_out, "state_out")
    cin, cout = state_in.c(), state_out.c()
    st = _lib.pond_stats() if stats else None
    _lib.check(lib.pond_step(C.byref(cfg.c()), C.byref(cin), C.byref(cout), int(nsteps),
                             _stream_ptr(state_in.f.device), C.byref(st) if stats else None))
    if stats:
        return state_out, {"nonconverged": st.nonconverged, "bad_state": st.bad_state,
                           "max_iters": st.max_iters, "mean_iters": st.mean_iters,
                           "iter_hist": [int(v) for v in st.iter_hist]}
    return state_out, None


def step_noalloc(cfg: PondConfig, state_in: PondState, state_out: PondState,
                 nsteps: int = 1, stats: bool = False):
    """pond_step_noalloc: pond_step on the library's fixed scratch (no device
    allocation by the library; both states are the caller's).  Returns
    (state_out, stats_dict or None)."""
    lib = _lib.load()
    _check_state(cfg, state_in, "state_in")
    _check_state(cfg, state_out, "state_out")
    cin, cout = state_in.c(), state_out.c()
    st = _lib.pond_stats() if stats else None
    _lib.check(lib.pond_step_noalloc(C.byref(cfg.c()), C.byref(cin), C.byref(cout), int(nsteps),
                                     _stream_ptr(state_in.f.device),
                                     C.byref(st) if stats else None))
    if stats:
        return state_out, {"nonconverged": st.nonconverged, "bad_state": st.bad_state,
                           "max_iters": st.max_iters, "mean_iters": st.mean_iters,
                           "iter_hist": [int(v) for v in st.iter_hist]}
    return state_out, None


def moments(cfg: PondConfig, state: PondState, raw: bool = False):
    """pond_moments.  Returns (rho, ux, uy, T[, Mmn]) as float64 device tensors."""
    lib = _lib.load()
    _check_state(cfg, state, "state")
    dev = state.f.device
    outs = [torch.empty((cfg.ny, cfg.nx), dtype=torch.float64, device=dev) for _ in range(4)]
    M = torch.empty((cfg.Q, cfg.ny, cfg.nx), dtype=torch.float64, device=dev) if raw else None
    cs = state.c()
    _lib.check(lib.pond_moments(C.byref(cfg.c()), C.byref(cs), *[o.data_ptr() for o in outs],
                                M.data_ptr() if raw else None, _stream_ptr(dev)))
    return (*outs, M) if raw else tuple(outs)


def workspace_bytes(cfg: PondConfig, op: int = POND_OP_STEP_ADJOINT) -> int:
    """pond_workspace_bytes: caller workspace of an operation."""
    n = C.c_int64(0)
    _lib.check(_lib.load().pond_workspace_bytes(C.byref(cfg.c()), int(op), C.byref(n)))
    return int(n.value)


def step_adjoint(cfg: PondConfig, state_in: PondState, state_out: PondState,
                 adj_f: torch.Tensor, adj_g: torch.Tensor, adj_tau: torch.Tensor | None = None,
                 workspace: torch.Tensor | None = None):
    """pond_step_adjoint: cotangents at t - dt from cotangents (adj_f, adj_g) at t.

    Returns (adj_f_in, adj_g_in); adds d<adj, out>/dtau into adj_tau (a 1-element
    float64 device tensor) when given.  `workspace` is a uint8 device tensor of
    at least workspace_bytes(cfg) bytes (allocated here when not given).
    """
    lib = _lib.load()
    _check_state(cfg, state_in, "state_in")
    _check_state(cfg, state_out, "state_out")
    dev = state_in.f.device
    _require(adj_f, (cfg.Q, cfg.ny, cfg.nx), torch.float64, "adj_f")
    _require(adj_g, (3, cfg.ny, cfg.nx), torch.float64, "adj_g")
    a_in_f = torch.empty_like(adj_f)
    a_in_g = torch.empty_like(adj_g)
    if adj_tau is not None:
        _require(adj_tau, (1,), torch.float64, "adj_tau")
    if workspace is None:
        workspace = torch.empty(workspace_bytes(cfg), dtype=torch.uint8, device=dev)
    if not workspace.is_cuda or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 device tensor")
    s_in, s_out = state_in.c(), state_out.c()
    a_out = _lib.pond_state(adj_f.data_ptr(), adj_g.data_ptr(), None)
    a_in = _lib.pond_state(a_in_f.data_ptr(), a_in_g.data_ptr(), None)
    _lib.check(lib.pond_step_adjoint(C.byref(cfg.c()), C.byref(s_in), C.byref(s_out),
                                     C.byref(a_out), C.byref(a_in),
                                     adj_tau.data_ptr() if adj_tau is not None else None,
                                     workspace.data_ptr(), workspace.numel(), _stream_ptr(dev)))
    return a_in_f, a_in_g


def init_adjoint(cfg: PondConfig, adj_f: torch.Tensor, adj_g: torch.Tensor):
    """pond_init_adjoint: (adj_rho, adj_ux, adj_uy, adj_T) from the cotangents
    of an initial state (f, g) = pond_init(rho, u, T)."""
    lib = _lib.load()
    dev = adj_f.device
    _require(adj_f, (cfg.Q, cfg.ny, cfg.nx), torch.float64, "adj_f")
    _require(adj_g, (3, cfg.ny, cfg.nx), torch.float64, "adj_g")
    outs = [torch.empty((cfg.ny, cfg.nx), dtype=torch.float64, device=dev) for _ in range(4)]
    _lib.check(lib.pond_init_adjoint(C.byref(cfg.c()), adj_f.data_ptr(), adj_g.data_ptr(),
                                     *[o.data_ptr() for o in outs], _stream_ptr(dev)))
    return tuple(outs)


def tape_bytes(cfg: PondConfig) -> int:
    """pond_tape_bytes: size of one recorded step's pass history."""
    n = C.c_int64(0)
    _lib.check(_lib.load().pond_tape_bytes(C.byref(cfg.c()), C.byref(n)))
    return int(n.value)


def step_record(cfg: PondConfig, state_in: PondState, state_out: PondState | None = None,
                tape: torch.Tensor | None = None):
    """pond_step_record: one step that also records its pass history.

    Returns (state_out, tape); tape is a uint8 device tensor of tape_bytes(cfg)
    bytes (allocated when not given)."""
    lib = _lib.load()
    _check_state(cfg, state_in, "state_in")
    dev = state_in.f.device
    if state_out is None:
        state_out = empty_state(cfg, dev)
    _check_state(cfg, state_out, "state_out")
    if state_out.iters is None:
        raise ValueError("step_record: state_out.iters is required")
    nb = tape_bytes(cfg)
    if tape is None:
        tape = torch.empty(nb, dtype=torch.uint8, device=dev)
    _require(tape, (nb,), torch.uint8, "tape")
    cin, cout = state_in.c(), state_out.c()
    _lib.check(lib.pond_step_record(C.byref(cfg.c()), C.byref(cin), C.byref(cout),
                                    tape.data_ptr(), _stream_ptr(dev)))
    return state_out, tape


def step_adjoint_recorded(cfg: PondConfig, state_in: PondState, state_out: PondState,
                          tape: torch.Tensor, adj_f: torch.Tensor, adj_g: torch.Tensor,
                          adj_tau: torch.Tensor | None = None):
    """pond_step_adjoint_recorded: step_adjoint about a step_record step."""
    lib = _lib.load()
    _check_state(cfg, state_in, "state_in")
    _check_state(cfg, state_out, "state_out")
    _require(tape, (tape_bytes(cfg),), torch.uint8, "tape")
    _require(adj_f, (cfg.Q, cfg.ny, cfg.nx), torch.float64, "adj_f")
    _require(adj_g, (3, cfg.ny, cfg.nx), torch.float64, "adj_g")
    if adj_tau is not None:
        _require(adj_tau, (1,), torch.float64, "adj_tau")
    a_in_f = torch.empty_like(adj_f)
    a_in_g = torch.empty_like(adj_g)
    s_in, s_out = state_in.c(), state_out.c()
    a_out = _lib.pond_state(adj_f.data_ptr(), adj_g.data_ptr(), None)
    a_in = _lib.pond_state(a_in_f.data_ptr(), a_in_g.data_ptr(), None)
    _lib.check(lib.pond_step_adjoint_recorded(
        C.byref(cfg.c()), C.byref(s_in), C.byref(s_out), tape.data_ptr(), C.byref(a_out),
        C.byref(a_in), adj_tau.data_ptr() if adj_tau is not None else None,
        _stream_ptr(state_in.f.device)))
    return a_in_f, a_in_g


def abi_version() -> int:
    return _lib.load().pond_abi_version()
