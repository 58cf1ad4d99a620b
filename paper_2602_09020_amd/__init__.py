"""MI355X (gfx950) hot path of the Clifford-fullstate hybrid simulator.

``cfh``     ctypes binding of libcfh (the C ABI in include/cfh.h).
``hybrid``  thin handle classes over it (Frame, Plan, Hamiltonian) and the
            torch.autograd.Function whose backward is the library's adjoint.
``build``   compiles libcfh.so in-tree with hipcc for gfx950.
"""
from . import cfh  # noqa: F401

__all__ = ["cfh"]
