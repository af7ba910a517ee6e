"""MI355X-native long-characteristics transport sweep (HIP for gfx950).

The compute path is the C ABI of ``liblc.so`` (declared in ``include/lc.h``);
``paper_2305_11998_amd.lc`` is its Python binding and ``driver`` runs whole
problems through it with PyTorch device memory.
"""
from . import lc  # noqa: F401  (raises ImportError when the library is not built)
