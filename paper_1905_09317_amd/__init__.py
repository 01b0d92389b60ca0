"""MI355X (gfx950) implementation of the Cell2Fire fire-growth hot path.

The simulation runs in libc2f.so (hand-written HIP kernels behind the C ABI
of include/c2f.h); this package only marshals arguments.
"""
from .api import C2FError, Request, Simulator, fbp_coefficients, fbp_crown_coefficients, request_for  # noqa: F401
