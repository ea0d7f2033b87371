"""Locally greedy convolutional coordinate descent (DICOD / LGCD) on MI355X.

The solver is the HIP library ``libdicod.so`` (C ABI in include/dicod.h);
this package only binds it.  See ``_binding`` for the entry points.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import (Context, DicodError, dicod_config, dicod_stats, lib,  # noqa: F401
                       TRACE_DTYPE, LIB_PATH)
