"""MI355X-native particle-mesh step for AQUAL MOND (arXiv 2312.02968).

The compute path is the HIP library ``libmondpm.so`` (C ABI in
``include/mondpm.h``); ``mondpm`` is its thin Python binding.
"""
from . import mondpm  # noqa: F401
from .mondpm import (Ctx, aqual_solve, interp_push, pm_create, pm_deposit, pm_destroy,  # noqa: F401
                     pm_diagnostics, pm_fft_c2r, pm_fft_r2c, pm_spectrum_pitch, pm_step,
                     pm_workspace_bytes, smooth_accel)
