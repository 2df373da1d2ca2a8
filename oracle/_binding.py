"""ctypes marshalling for the oracle library (no arithmetic of the method here)."""
import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpond_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("POND_ORACLE_LIBRARY", _LIB_PATH)  # another build of the same source
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        from .build_oracle import build
        build()
    lib = C.CDLL(path)
    I, D = C.c_int, C.c_double
    lib.oracle_lattice.argtypes = [I, _dp, _dp, _dp]
    lib.oracle_transfer_1d.argtypes = [I, D, D, D, D, _dp]
    lib.oracle_transfer_2d.argtypes = [I, D, D, D, D, D, D, _dp]
    lib.oracle_lagrange_weight.argtypes = [D, I]
    lib.oracle_lagrange_weight.restype = D
    lib.oracle_init.argtypes = [I, I, I, _dp, _dp, _dp, _dp, _dp, _dp]
    cfg = [I, I, I, I, I, I, I, I, I]  # q nx ny iso bcx bcy max fixed seed
    lib.oracle_step.argtypes = cfg + [D, D, D, _dp, _dp, _dp, _dp, _ip, _ip]
    lib.oracle_step_nodes.argtypes = cfg + [D, D, D, _dp, _dp, C.c_longlong, _lp, _dp, _dp, _ip, _ip]
    lib.oracle_moments.argtypes = [I, I, I, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_init_cs.argtypes = [I, I, I] + [_dp] * 12
    lib.oracle_step_cs.argtypes = cfg + [D, D, D, D] + [_dp] * 8 + [_ip, _ip]
    lib.oracle_moments_cs.argtypes = [I, I, I] + [_dp] * 12
    lib.oracle_num_threads.restype = I
    lib.oracle_set_num_threads.argtypes = [I]
    lib.oracle_set_num_threads.restype = I
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclasses.dataclass
class OracleConfig:
    """Parameters of one step (defaults: the paper's tolerances, App. E)."""
    q: int = 4
    isothermal: int = 0
    bc_x: int = 0  # 0 periodic, 1 zero gradient
    bc_y: int = 0
    max_iter: int = 20
    fixed_iter: int = 0
    seed_mode: int = 0
    tau: float = 0.6
    eps_abs: float = 1e-12
    eps_rel: float = 1e-10

    def _ints(self, nx, ny):
        return [self.q, nx, ny, self.isothermal, self.bc_x, self.bc_y, self.max_iter,
                self.fixed_iter, self.seed_mode]


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> int:
    """Threads for the following oracle calls; returns the previous count."""
    return _load().oracle_set_num_threads(int(n))


def lattice(q: int = 4):
    """Return (c, w, T_L) for the 1-D speed set (q = 4: D2Q16 factor, q = 3: D2Q9 factor)."""
    c = np.zeros(4)
    w = np.zeros(4)
    TL = C.c_double()
    if _load().oracle_lattice(q, _p(c), _p(w), C.byref(TL)) != 0:
        raise ValueError("unsupported q")
    return c[:q].copy(), w[:q].copy(), TL.value


def transfer_1d(q, u_src, T_src, u_dst, T_dst):
    G = np.zeros(q * q)
    _load().oracle_transfer_1d(q, float(u_src), float(T_src), float(u_dst), float(T_dst), _p(G))
    return G.reshape(q, q)


def transfer_2d(q, src, dst):
    """Explicit Q x Q transfer matrix; src/dst = (u_x, u_y, T)."""
    Q = q * q
    G = np.zeros(Q * Q)
    _load().oracle_transfer_2d(q, *map(float, src), *map(float, dst), _p(G))
    return G.reshape(Q, Q)


def lagrange_weight(t, n):
    return _load().oracle_lagrange_weight(float(t), int(n))


def init(rho, ux, uy, T, q=4):
    rho, ux, uy, T = map(_c64, (rho, ux, uy, T))
    ny, nx = rho.shape
    f = np.zeros((q * q, ny, nx))
    g = np.zeros((3, ny, nx))
    _load().oracle_init(q, nx, ny, _p(rho), _p(ux), _p(uy), _p(T), _p(f), _p(g))
    return f, g


def step(f, g, cfg: OracleConfig):
    """One step over the grid. Returns (f_out, g_out, iters, status)."""
    f, g = _c64(f), _c64(g)
    _, ny, nx = g.shape
    fo = np.empty_like(f)
    go = np.empty_like(g)
    it = np.zeros((ny, nx), np.int32)
    st = np.zeros((ny, nx), np.int32)
    _load().oracle_step(*cfg._ints(nx, ny), cfg.tau, cfg.eps_abs, cfg.eps_rel, _p(f), _p(g),
                        _p(fo), _p(go), it.ctypes.data_as(_ip), st.ctypes.data_as(_ip))
    return fo, go, it, st


def step_nodes(f, g, cfg: OracleConfig, nodes):
    """One step evaluated only at flat node indices ``nodes`` (y*nx + x).

    Returns (f_sel [Q, n], g_sel [3, n], iters [n], status [n]).
    """
    f, g = _c64(f), _c64(g)
    _, ny, nx = g.shape
    sel = np.ascontiguousarray(nodes, dtype=np.int64)
    n = sel.size
    Q = cfg.q * cfg.q
    fo = np.empty((Q, n))
    go = np.empty((3, n))
    it = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    _load().oracle_step_nodes(*cfg._ints(nx, ny), cfg.tau, cfg.eps_abs, cfg.eps_rel, _p(f), _p(g),
                              n, sel.ctypes.data_as(_lp), _p(fo), _p(go), it.ctypes.data_as(_ip),
                              st.ctypes.data_as(_ip))
    return fo, go, it, st


def moments(f, g, q=4, with_raw=False):
    """Return (rho, ux, uy, T[, Mmn]) of a state."""
    f, g = _c64(f), _c64(g)
    _, ny, nx = g.shape
    rho, ux, uy, T = (np.empty((ny, nx)) for _ in range(4))
    M = np.empty((q * q, ny, nx)) if with_raw else None
    _load().oracle_moments(q, nx, ny, _p(f), _p(g), _p(rho), _p(ux), _p(uy), _p(T), _p(M))
    if with_raw:
        return rho, ux, uy, T, M
    return rho, ux, uy, T


def _split(z):
    z = np.asarray(z, dtype=np.complex128)
    return np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)


def init_cs(rho, ux, uy, T, q=4):
    """Complex-valued equilibrium initialisation (complex-step differentiation)."""
    parts = [_split(a) for a in (rho, ux, uy, T)]
    ny, nx = parts[0][0].shape
    fr, fi = np.zeros((q * q, ny, nx)), np.zeros((q * q, ny, nx))
    gr, gi = np.zeros((3, ny, nx)), np.zeros((3, ny, nx))
    args = [_p(a) for pr in parts for a in pr]
    _load().oracle_init_cs(q, nx, ny, *args, _p(fr), _p(fi), _p(gr), _p(gi))
    return fr + 1j * fi, gr + 1j * gi


def step_cs(f, g, cfg: OracleConfig, tau=None):
    """One step in complex arithmetic; ``tau`` may be complex."""
    fr, fi = _split(f)
    gr, gi = _split(g)
    _, ny, nx = gr.shape
    tau = complex(cfg.tau if tau is None else tau)
    for_, foi = np.empty_like(fr), np.empty_like(fr)
    gor, goi = np.empty_like(gr), np.empty_like(gr)
    it = np.zeros((ny, nx), np.int32)
    st = np.zeros((ny, nx), np.int32)
    _load().oracle_step_cs(*cfg._ints(nx, ny), tau.real, tau.imag, cfg.eps_abs, cfg.eps_rel,
                           _p(fr), _p(fi), _p(gr), _p(gi), _p(for_), _p(foi), _p(gor), _p(goi),
                           it.ctypes.data_as(_ip), st.ctypes.data_as(_ip))
    return for_ + 1j * foi, gor + 1j * goi, it, st


def moments_cs(f, g, q=4):
    fr, fi = _split(f)
    gr, gi = _split(g)
    _, ny, nx = gr.shape
    outs = [np.empty((ny, nx)) for _ in range(8)]
    _load().oracle_moments_cs(q, nx, ny, _p(fr), _p(fi), _p(gr), _p(gi), *[_p(o) for o in outs])
    return tuple(outs[2 * k] + 1j * outs[2 * k + 1] for k in range(4))
