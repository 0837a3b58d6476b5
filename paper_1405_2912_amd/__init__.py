"""MI355X (gfx950) heterogeneity-aware majority voter.

The C ABI is declared in ``include/ftv.h`` and implemented by ``libftv.so``
(hand-written HIP kernels); this package is its thin Python binding.
"""
from .ftv import *  # noqa: F401,F403
from .ftv import load  # noqa: F401
