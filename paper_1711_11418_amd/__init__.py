"""MI355X-native many-variable VMC hot path (arXiv:1711.11418).

The compute lives in libmvmc.so (HIP kernels for gfx950 behind the C ABI in
include/mvmc.h); ``binding`` marshals arguments from Python/PyTorch.
"""
from .binding import MVMC, MVMCError, load, make_config, query_layout, query_sizes

__all__ = ["MVMC", "MVMCError", "load", "make_config", "query_layout", "query_sizes"]
