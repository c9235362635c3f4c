"""MI355X-native exponential stepper for complex Ginzburg--Landau equations.

The work is done by ``libcgl.so`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/cgl.h``); ``paper_2403_02816_amd.cgl`` is its Python
binding.  Build with ``python -m paper_2403_02816_amd.build``.
"""
from . import _lib  # noqa: F401  (declarations only; the library loads on first use)

__all__ = ["cgl", "build"]
