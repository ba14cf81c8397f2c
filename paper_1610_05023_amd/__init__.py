"""MI355X time stepper for nodal DG with high-order absorbing boundary
conditions and corner/edge compatibility (arXiv:1610.05023).

The product is libdghabc.so (C ABI in include/dghabc.h: C++ host setup and
hand-written HIP kernels for gfx950); ``binding`` is its thin ctypes
binding, with PyTorch supplying device memory and streams.
"""
from .binding import Solver, DghError, load, ARRAYS, COUNTS, BC  # noqa: F401
