"""Particles-on-Demand (arXiv:1806.05089) time step for AMD MI355X (gfx950).

The product is the C-ABI library ``libpond.so`` (HIP kernels, declared in
``include/pond.h``).  ``pond`` is its thin Python binding over torch device
tensors, ``autograd`` a checkpointed torch.autograd.Function over the
hand-written adjoint, and ``workloads`` the seeded synthetic input fields.
Importing the package does not load the library; the first call does, and
fails loudly if it is missing.
"""
__all__ = ["pond", "workloads", "autograd"]
