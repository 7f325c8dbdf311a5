"""grwave: backward generalized-ray wave-optical path tracing on AMD Instinct MI355X.

Hand-written HIP kernels for gfx950 behind the C ABI of ``libgrwave.so``
(``include/grwave.h``); this package is the thin Python binding over it.
"""

from ._lib import GR_BSDF_PLAIN, GR_BSDF_SURROGATE_BF16, GR_BSDF_SURROGATE_FP8, GrError  # noqa: F401
from .renderer import Renderer  # noqa: F401
