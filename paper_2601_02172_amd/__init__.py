"""MI355X-native X-FFT solver for periodic linear-elastic cell problems.

The numerical work runs in ``libxfft.so`` (hand-written HIP for gfx950, C ABI
in ``include/xfft.h``); this package only marshals arguments.
"""

from .xfft import (Problem, XfftError, batch_effective_stiffness, default_options, LIB_PATH, EXPORTS,
                   XFFT_OK, XFFT_NOT_CONVERGED, XFFT_EINVAL, XFFT_ENOMEM, XFFT_EDEVICE, XFFT_EBREAKDOWN)

__all__ = ["Problem", "XfftError", "batch_effective_stiffness", "default_options", "LIB_PATH", "EXPORTS",
           "XFFT_OK", "XFFT_NOT_CONVERGED", "XFFT_EINVAL", "XFFT_ENOMEM", "XFFT_EDEVICE", "XFFT_EBREAKDOWN"]
