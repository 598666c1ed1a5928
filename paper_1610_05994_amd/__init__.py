"""MI355X-native pointerless wavelet-tree construction (HIP for gfx950).

The product is the C-ABI library ``libwtree.so`` (declared in
``include/wtree.h``); ``wtree`` is its thin ctypes binding.
"""
from . import wtree  # noqa: F401
from .wtree import Tree, build, build_batch, to_device  # noqa: F401
