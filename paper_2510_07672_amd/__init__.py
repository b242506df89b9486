"""MI355X (gfx950) Parareal fine propagator for the Allen-Cahn equations.

The computation lives in libpr.so (HIP kernels behind the C ABI of
include/pr.h); `api` is its thin torch binding and `build` compiles it.
Importing this package loads nothing: the library is opened on first use
and a missing build is an error.
"""

__all__ = ["api", "build", "synth"]
