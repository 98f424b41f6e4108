"""MI355X (gfx950) library for the Kuramoto model on graphs with localised order parameters.

The compute path is the C-ABI shared library ``libkur.so`` (HIP kernels, include/kur.h);
``kur.Kuramoto`` is its thin Python binding.
"""
from .buildlib import build  # noqa: F401
from .kur import Kuramoto, KurError, lib  # noqa: F401
