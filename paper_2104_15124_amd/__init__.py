"""MI355X-native builder of self-tuning variable-bandwidth kernel matrices.

The sparse kernel matrix approximating the Kolmogorov operator L_{c,psi} of
Davis & Giannakis (arXiv 2104.15124) is assembled by hand-written HIP kernels
for gfx950 behind the C ABI in ``include/kvb.h``; ``kvb`` is its Python binding.
"""
import importlib

__all__ = ["kvb"]


def __getattr__(name):
    if name == "kvb":
        return importlib.import_module(__name__ + ".kvb")
    raise AttributeError(name)
