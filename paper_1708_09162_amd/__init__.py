"""MI355X-native fast isogeometric single-layer BEM (Laplace / Helmholtz).

The compute path lives in the C-ABI shared library ``libigabem.so`` built
from ``csrc/``; ``igabem`` is its thin ctypes binding.  Importing this package
does not load the library: ``from paper_1708_09162_amd import igabem`` does.
"""
__all__ = ["igabem", "workloads"]
