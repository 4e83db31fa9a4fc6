"""MI355X-native coupled Yee + LLG (Maxwell-Landau-Lifshitz-Gilbert) FDTD step.

The hot path is the HIP library ``libmpx.so`` built from ``csrc/`` for gfx950;
``mpx`` is its ctypes binding.
"""
from . import mpx  # noqa: F401
