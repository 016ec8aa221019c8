"""MI355X (gfx950) implementation of the adaptive product-convolution apply
of Alger, Rao, Myers, Bui-Thanh and Ghattas (arXiv 1805.06018).

The product is the C-ABI library libpc.so (include/pc.h); this package holds
its HIP/C++ sources (csrc/), the build step (build.py) and a thin ctypes
binding (_lib.py, imported lazily so that the build can run without it).
"""


def load():
    """Import the binding; raises ImportError if libpc.so is not built."""
    from . import _lib
    return _lib
