"""LFA singular value decomposition of periodic stride-1 convolutions on
AMD MI355X (gfx950): HIP kernels behind a C ABI (include/lfa.h), with a thin
PyTorch binding.  Build the library with ``python -m paper_2506_05617_amd.build``.
"""

from .lfa import (  # noqa: F401
    GraphStep,
    LayerSpec,
    Plan,
    SigmaTopK,
    crystal_layer,
    crystal_weights,
    sigma_sum,
    sigma_topk,
    svd,
    symbols,
)
from ._lib import LfaError, load  # noqa: F401
