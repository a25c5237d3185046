"""MI355X-native particle-mesh step with compressed particles (arXiv:1611.01545).

The compute path is libpm.so (HIP kernels for gfx950 behind the C ABI in
include/pm.h); this package is its Python binding.
"""

from .pm import CompressedSpecies, FloatSpecies, G_UNIT, PMContext, widths_word  # noqa: F401
