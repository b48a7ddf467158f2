"""MI355X-native hybrid fluid-kinetic laser-plasma step (arXiv 2510.11174).

The compute path is the C-ABI shared library built from ``csrc/`` for gfx950
(``libhk_f32.so`` / ``libhk_f64.so``); ``hk`` is its thin ctypes binding.
Importing the package does not load the library: ``hk.Sim`` does, and raises
if it has not been built.
"""
from . import configs  # noqa: F401

__all__ = ["configs"]
