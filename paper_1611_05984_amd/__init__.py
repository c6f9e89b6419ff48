"""MI355X-native time step of the Celeris extended-Boussinesq wave solver.

The solver runs in hand-written HIP kernels behind the C ABI declared in
``include/wavestep.h`` (``libwavestep.so``).  ``wavestep`` is the thin ctypes
binding (PyTorch supplies device memory and streams); ``workloads`` draws the
seeded synthetic inputs.  Importing this package loads nothing; the binding
loads the library on first use and raises if it is missing.
"""
__all__ = ["wavestep", "workloads"]
