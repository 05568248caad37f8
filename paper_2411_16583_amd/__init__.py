"""MI355X-native Fourier-Galerkin chemo-mechanical solver core.

The hot path (FFTs, projection, tangent contraction, Krylov updates,
phase-field and Fick operators) is hand-written HIP in ``csrc/`` compiled
into ``libfgfft.so``; ``fgfft`` is its ctypes binding and ``driver`` the
staggered time-stepping loop built on the C ABI.
"""
from .fgfft import Batch, FgError, Plan, load_library, make_opts  # noqa: F401
