"""MI355X-native batched plane-wave sphere<->grid 3D FFT.

The transform path runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in include/fftb.h; `Plan` is a thin binding over it. Importing the
package does not load the library; creating a plan does, and fails loudly if
libfftb.so has not been built.
"""
from .fftb import (  # noqa: F401
    Plan, FftbError, lib, LIB_PATH, EXPORTS,
    FFTB_OK, FFTB_ERR_INVALID, FFTB_ERR_UNSUPPORTED, FFTB_ERR_NOMEM, FFTB_ERR_HIP,
    FFTB_C128, FFTB_C64,
    PLAN_PLAIN, PLAN_BATCHED, PLAN_AUTOTUNE, PLAN_GRAPH, PLAN_HOST_ONLY, PLAN_MFMA,
)
