"""Plain FP64 CPU oracle of the Particles-on-Demand time step (arXiv:1806.05089).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only code allowed to import this package.  The
product (the HIP library and its Python binding) never imports it.

The arithmetic lives in ``pond_oracle.cpp`` (plain loops, explicit linear
solves for the transfer matrix of eq. (4)); this module only marshals numpy
arrays through ctypes.  ``riemann`` holds the exact Riemann solution used to pin
the thermal step (a textbook closed form, not part of the method).
"""
from ._binding import (  # noqa: F401
    lattice,
    transfer_1d,
    transfer_2d,
    lagrange_weight,
    init,
    step,
    step_nodes,
    moments,
    init_cs,
    step_cs,
    moments_cs,
    num_threads,
    set_num_threads,
    OracleConfig,
    library_path,
)
