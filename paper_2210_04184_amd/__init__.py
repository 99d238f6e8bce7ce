"""MI355X (gfx950) implementation of the guided nonlocal patch-regularised fusion ADMM
(arXiv 2210.04184): a HIP library with a C ABI (include/nlpr.h) and a thin ctypes binding."""
from . import nlpr  # noqa: F401
from .nlpr import Plan, fuse, NlprError  # noqa: F401
