"""MI355X-native FFT binned angular bispectrum estimator for gridded visibilities
(Gill, Bharadwaj, Ali & Elahi 2024).  The compute path is libabs.so: hand-written
HIP kernels for gfx950 behind the C ABI of include/abs.h.  This package is the thin
Python binding over it."""
from ._lib import (ALL_MFMA, ALLOW_DC, ALLOW_WRAP, BEAM_GAUSS, BEAM_MWA, BEAM_NONE, BF16X3, C64, C128,  # noqa: F401
                   EVERY_LEVEL, FP16X3, FP32, GAUSS7, NEAREST, W_GIVEN, W_INV_COUNT, W_UNIT, AbsError, lib)
from .plan import BaselineSet, Plan, ensemble, simulate  # noqa: F401
