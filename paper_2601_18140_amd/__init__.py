"""MI355X (gfx950) implementation of the RTeAAL Sim layer cascade.

`rteaal` is the ctypes binding of librteaal.so (built by `build.py`); its
functions carry the names of the C entry points in include/rteaal.h.
"""
from . import rteaal  # noqa: F401
from .rteaal import *  # noqa: F401,F403
from .rteaal import __all__  # noqa: F401
