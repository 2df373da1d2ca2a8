"""Seeded synthetic inputs: macroscopic fields (rho, u_x, u_y, T) and step parameters.

This module holds no arithmetic of the method.  It only writes down the initial
flow fields of the workloads as closed forms or seeded draws, so that the HIP
path and the CPU oracle can be fed identical inputs.  Arrays are float64, shape
[ny][nx]; x is the column (node) index, y the row index, lattice units with
dx = dt = 1.  The lattice temperature of the D2Q16 speed set is T_L = 1.

Workloads (all synthetic; the paper uses no dataset):

* ``taylor_green``: periodic Taylor-Green vortex of App. D (Green-Taylor
  vortex), u_x = -(u0/sqrt2) cos kx sin ky, u_y = (u0/sqrt2) sin kx cos ky,
  k = 2 pi / N, isothermal.
* ``sod``: quasi-1-D shock tube, left/right (rho, p) = (1, 1) / (0.125, 0.1),
  u = 0, diaphragm at x = nx/2 - 1/2, temperature T = s p / rho with the scale
  s (default 0.25) so that the waves stay inside the tube.  rho and p change
  across the diaphragm as 1/2 (1 - tanh((x - x_d) / width)) with width = 1 node
  (width = 0: a sharp jump, at which the predictor-corrector iteration of the
  first node downstream diverges).
* ``mach5``: uniform flow U = (5 sqrt(T), 0) at T = T_L with an i.i.d.
  Gaussian density perturbation of amplitude 1e-3.
* ``compressible_taylor_green``: thermal Taylor-Green vortex at Mach 0.5 plus
  an i.i.d. Gaussian velocity perturbation 0.01 u0 N(0, 1).
* ``riemann2d``: four-quadrant 2-D Riemann problem; per quadrant rho ~
  U[0.5, 1.5], p ~ U[0.3, 1.5], T = p / rho, u_x, u_y ~ U[-0.8, 0.8] sqrt(T).

D2Q9 experiments of the paper (lattice temperature T_L = 1/3):

* ``shear_wave``: isothermal plane shear wave whose wave vector is tilted by
  pi/4: transverse velocity A sin(2 pi (x + y) / N) along (-1, 1)/sqrt2,
  advection Ma_a sqrt(T) along the wave vector (1, 1)/sqrt2, on an N x N
  periodic grid (wavelength N / sqrt2 along the diagonal).
* ``sound_pulse``: gas at rest or advected (u = Ma_a sqrt(T)) with a Gaussian
  pressure disturbance of amplitude 1e-3 at uniform density, 1-D periodic.
* ``thermal_wave``: rho = rho0 + A sin(2 pi x / L) at uniform pressure
  p = rho0 T0, advected with u = Ma_a sqrt(2 T0), 1-D periodic.
* ``vortex``: isothermal vortex u_phi(r) = Ma_v c r exp((1 - r^2) / 2),
  r = r'/R, c = sqrt(2 T), with the density that balances the centrifugal
  force at uniform T, rho = exp(-Ma_v^2 exp(1 - r^2)), advected with
  U = Ma_a c along x, periodic.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    tau: float
    isothermal: int
    bc_x: int  # 0 periodic, 1 zero gradient
    bc_y: int
    steps: int
    meta: dict

    @property
    def shape(self):
        return self.rho.shape


def _grid(nx, ny):
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    return np.meshgrid(x, y)  # X[y, x], Y[y, x]


def taylor_green(N: int = 32, mach: float = 0.05, T0: float = 1.0, rho0: float = 1.0,
                 tau: float = 0.6, steps: int = 200, isothermal: int = 1) -> Workload:
    X, Y = _grid(N, N)
    k = 2.0 * math.pi / N
    u0 = mach * math.sqrt(T0)
    a = u0 / math.sqrt(2.0)
    ux = -a * np.cos(k * X) * np.sin(k * Y)
    uy = a * np.sin(k * X) * np.cos(k * Y)
    return Workload("taylor_green", np.full((N, N), rho0), ux, uy, np.full((N, N), T0), tau,
                    isothermal, 0, 0, steps, {"N": N, "u0": u0, "k": k, "T0": T0})


def sod(nx: int = 1024, ny: int = 4, scale: float = 0.25, tau: float = 0.52,
        steps: int = 400, width: float = 1.0) -> Workload:
    x = np.arange(nx, dtype=np.float64)
    xd = nx // 2 - 0.5
    if width > 0:
        left = 0.5 * (1.0 - np.tanh((x - xd) / width))
    else:
        left = (x < xd).astype(np.float64)
    rho_row = 0.125 + (1.0 - 0.125) * left
    p_row = 0.1 + (1.0 - 0.1) * left
    rho = np.tile(rho_row, (ny, 1))
    T = np.tile(scale * p_row / rho_row, (ny, 1))
    z = np.zeros((ny, nx))
    return Workload("sod", rho, z.copy(), z.copy(), T, tau, 0, 1, 0, steps,
                    {"scale": scale, "x_diaphragm": xd, "width": width,
                     "left": (1.0, 0.0, 1.0), "right": (0.125, 0.0, 0.1)})


def mach5(N: int = 256, mach: float = 5.0, T0: float = 1.0, amp: float = 1e-3, seed: int = 0,
          tau: float = 0.6, steps: int = 1000, U: float | None = None) -> Workload:
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.standard_normal((N, N))
    Ux = mach * math.sqrt(T0) if U is None else U
    return Workload("mach5", rho, np.full((N, N), Ux), np.zeros((N, N)), np.full((N, N), T0),
                    tau, 0, 0, 0, steps, {"U": Ux, "seed": seed, "amp": amp})


def compressible_taylor_green(N: int = 128, mach: float = 0.5, T0: float = 1.0, seed: int = 1,
                              pert: float = 0.01, tau: float = 0.6, steps: int = 200) -> Workload:
    X, Y = _grid(N, N)
    k = 2.0 * math.pi / N
    u0 = mach * math.sqrt(T0)
    a = u0 / math.sqrt(2.0)
    rng = np.random.default_rng(seed)
    ux = -a * np.cos(k * X) * np.sin(k * Y) + pert * u0 * rng.standard_normal((N, N))
    uy = a * np.sin(k * X) * np.cos(k * Y) + pert * u0 * rng.standard_normal((N, N))
    return Workload("compressible_taylor_green", np.ones((N, N)), ux, uy, np.full((N, N), T0),
                    tau, 0, 0, 0, steps, {"u0": u0, "k": k, "seed": seed})


def riemann2d(N: int = 1024, seed: int = 3, tau: float = 0.55, steps: int = 2000,
              T_scale: float = 1.0) -> Workload:
    """Four-quadrant 2-D Riemann problem.  T_scale multiplies every temperature
    (velocities follow through sqrt(T), so the Mach numbers stay): 1 for D2Q16
    (T_L = 1), TL_D2Q9 for the same flow on D2Q9."""
    rng = np.random.default_rng(seed)
    # quadrant order: (lower-left, lower-right, upper-left, upper-right) in (y, x)
    q_rho = rng.uniform(0.5, 1.5, 4)
    q_p = rng.uniform(0.3, 1.5, 4)
    q_T = q_p / q_rho * T_scale
    q_ux = rng.uniform(-0.8, 0.8, 4) * np.sqrt(q_T)
    q_uy = rng.uniform(-0.8, 0.8, 4) * np.sqrt(q_T)
    h = N // 2
    quad = np.zeros((N, N), dtype=np.int64)
    quad[:h, h:] = 1
    quad[h:, :h] = 2
    quad[h:, h:] = 3
    return Workload("riemann2d", q_rho[quad], q_ux[quad], q_uy[quad], q_T[quad], tau, 0, 1, 1,
                    steps, {"seed": seed, "rho": q_rho.tolist(), "p": q_p.tolist(),
                            "ux": q_ux.tolist(), "uy": q_uy.tolist(), "T_scale": T_scale})


def uniform(nx: int, ny: int, rho: float = 1.0, ux: float = 0.0, uy: float = 0.0, T: float = 1.0,
            tau: float = 0.6, isothermal: int = 0) -> Workload:
    return Workload("uniform", np.full((ny, nx), rho), np.full((ny, nx), ux), np.full((ny, nx), uy),
                    np.full((ny, nx), T), tau, isothermal, 0, 0, 1, {})


def shifted(w: Workload, dux: float, duy: float = 0.0) -> Workload:
    """The same fields riding on an extra uniform velocity (dux, duy)."""
    return dataclasses.replace(w, name=w.name + "_shifted", ux=w.ux + dux, uy=w.uy + duy)


def random_smooth(nx: int, ny: int, seed: int = 0, mach: float = 0.3, T0: float = 1.0,
                  dT: float = 0.2, drho: float = 0.1, modes: int = 3, tau: float = 0.6) -> Workload:
    """Smooth random periodic fields (a few Fourier modes per field) for parity tests."""
    rng = np.random.default_rng(seed)
    X, Y = _grid(nx, ny)

    def field():
        out = np.zeros((ny, nx))
        for _ in range(modes):
            kx = rng.integers(-2, 3)
            ky = rng.integers(-2, 3)
            ph = rng.uniform(0, 2 * math.pi)
            out += rng.standard_normal() * np.cos(2 * math.pi * (kx * X / nx + ky * Y / ny) + ph)
        return out / math.sqrt(modes)

    rho = 1.0 + drho * np.tanh(field())
    T = T0 * (1.0 + dT * np.tanh(field()))
    ux = mach * math.sqrt(T0) * field()
    uy = mach * math.sqrt(T0) * field()
    return Workload("random_smooth", rho, ux, uy, T, tau, 0, 0, 0, 1, {"seed": seed})


TL_D2Q9 = 1.0 / 3.0


def shear_wave(N: int = 128, T: float = TL_D2Q9, mach_a: float = 0.0, nu: float = 0.02,
               A: float = 0.05) -> Workload:
    """Tilted shear wave; tau from nu = T (tau - 1/2)."""
    X, Y = _grid(N, N)
    ut = A * np.sin(2 * math.pi * (X + Y) / N)   # transverse, along (-1, 1)/sqrt2
    ul = mach_a * math.sqrt(T)                   # advection along (1, 1)/sqrt2
    r2 = 1.0 / math.sqrt(2.0)
    ux = r2 * (ul - ut)
    uy = r2 * (ul + ut)
    tau = 0.5 + nu / T
    return Workload("shear_wave", np.ones((N, N)), ux, uy, np.full((N, N), T), tau, 1, 0, 0, 0,
                    {"A": A, "k": 2 * math.pi * math.sqrt(2.0) / N, "nu": nu, "mach_a": mach_a})


def sound_pulse(nx: int = 512, T0: float = TL_D2Q9, mach_a: float = 0.0, amp: float = 1e-3,
                width: float = 4.0, tau: float = 0.6) -> Workload:
    """Pressure disturbance carried by the temperature at uniform density."""
    x = np.arange(nx, dtype=np.float64)
    x0 = nx / 2.0
    T = T0 * (1.0 + amp * np.exp(-((x - x0) / width) ** 2))
    U = mach_a * math.sqrt(T0)
    return Workload("sound_pulse", np.ones((1, nx)), np.full((1, nx), U), np.zeros((1, nx)),
                    T[None], tau, 0, 0, 0, 0, {"x0": x0, "U": U, "T0": T0})


def thermal_wave(L: int = 300, T0: float = TL_D2Q9, mach_a: float = 0.0, A: float = 1e-3,
                 rho0: float = 1.0, tau: float = 0.6) -> Workload:
    """Density wave at uniform pressure (an entropy wave); Ma_a = u / sqrt(2 T0)."""
    x = np.arange(L, dtype=np.float64)
    rho = rho0 + A * np.sin(2 * math.pi * x / L)
    T = rho0 * T0 / rho
    U = mach_a * math.sqrt(2.0 * T0)
    return Workload("thermal_wave", rho[None], np.full((1, L), U), np.zeros((1, L)), T[None], tau,
                    0, 0, 0, 0, {"k": 2 * math.pi / L, "U": U, "T0": T0, "A": A})


def vortex(N: int = 128, R: float = 10.0, mach_v: float = 0.8, mach_a: float = 0.0,
           T: float = TL_D2Q9, tau: float = 0.6) -> Workload:
    """Vortex of radius R at the grid centre; Ma_v and Ma_a relative to sqrt(2 T)."""
    X, Y = _grid(N, N)
    c = math.sqrt(2.0 * T)
    dx = (X - N / 2.0) / R
    dy = (Y - N / 2.0) / R
    r2 = dx * dx + dy * dy
    amp = mach_v * c * np.exp((1.0 - r2) / 2.0)   # u_phi / r
    ux = -amp * dy + mach_a * c
    uy = amp * dx
    rho = np.exp(-mach_v * mach_v * np.exp(1.0 - r2))
    return Workload("vortex", rho, ux, uy, np.full((N, N), T), tau, 0, 0, 0, 0,
                    {"R": R, "mach_v": mach_v, "mach_a": mach_a, "U": mach_a * c})
