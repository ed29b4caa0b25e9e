"""nbx: MI355X-native direct N-body force library (the GPU half of a GRAPE-style N-body code).

The computation lives in ``libnbx.so`` (HIP kernels for gfx950 behind the C ABI of
``include/nbx.h``); this package is its ctypes binding.  Build with
``python -m paper_1510_04068_amd.build``.
"""

from .nbx import *  # noqa: F401,F403
from .nbx import (  # noqa: F401
    EXPORTS,
    LIB_PATH,
    Context,
    NbxError,
    load,
)
