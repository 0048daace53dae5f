"""MI355X (gfx950) multigrid compact gas-kinetic scheme: Python binding of libcgks.

The binding only marshals arguments to the C ABI declared in include/cgks.h;
every step of the solver runs in the HIP library.  If libcgks.so has not been
built (``python -m paper_2509_06347_amd.build`` or ``__graft_entry__.build()``)
importing :mod:`paper_2509_06347_amd.cgks` raises ImportError: there is no
CPU fallback.
"""

__all__ = ["cgks"]
