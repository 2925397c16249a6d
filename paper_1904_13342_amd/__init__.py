"""MI355X-native known-operator CT layers (PYRO-NN, arXiv 1904.13342).

Hand-written HIP kernels for gfx950 behind the C ABI of include/pyrohip.h;
this package is the thin Python binding.  Importing it loads libpyrohip.so
and raises if the library has not been built.
"""
from ._lib import lib as _load_lib

_load_lib()

from .ops import *  # noqa: E402,F401,F403
from .ops import __all__ as _ops_all  # noqa: E402
from . import autograd  # noqa: E402,F401
from .corrector import LearnedCorrector, LearnedFilter2D  # noqa: E402,F401
from .iterative import TVReconstruction  # noqa: E402,F401

__all__ = list(_ops_all) + ["autograd", "LearnedCorrector", "LearnedFilter2D", "TVReconstruction"]
