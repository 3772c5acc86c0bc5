"""MI355X-native evaluator for pixelated multi-layer MoM inverse design
(arXiv 2412.17617): gather of active RWG rows and columns, batched dense
complex LU, S-parameters and figure of merit, all in gfx950 kernels behind the
C ABI of ``include/pxd.h``.  ``pxd`` is the Python binding.
"""

from . import pxd  # noqa: F401
