"""MI355X-native finite-volume hot path of arXiv 2203.00925 (Manapy).

``binding`` is the ctypes binding of libmifvm (include/mifvm.h); ``build``
compiles the library for gfx950.  Importing the binding requires the built
library; there is no CPU fallback.
"""
__all__ = ["binding", "build"]
