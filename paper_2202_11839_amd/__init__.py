"""MI355X-native LPP estimator of projected-tensor power-spectrum multipoles.

The estimator (Kurita & Takada, arXiv:2202.11839, Sec. III.A) runs in the HIP
kernels of ``liblpp.so`` behind the C ABI in ``include/lpp.h``; this package
is its thin Python binding.  Importing it does not load the library; the first
``Plan`` does, and fails loudly if ``liblpp.so`` has not been built.
"""
from ._lib import (LPP_ALL, LPP_DD, LPP_F32, LPP_F64, LPP_GD, LPP_MINUS, LPP_PLUS, LppError, Plan,  # noqa: F401
                   load, version, EXPORTS, LIB_PATH, template_plain, template_plain_noalloc, template_multipoles,
                   TEMPLATE_SERIES, window_coefficient, window_pairs, Mlp)
