"""GEEK's data pass on AMD Instinct MI355X (gfx950).

The method (Luo, Huang, Tung, arXiv 2106.10515) turns objects into LSH
buckets, finds seeds from similar buckets (SILK) and assigns every object once
to its nearest central vector.  The kernels live in ``libgeek.so`` (HIP, built
from ``csrc/``) behind the C ABI of ``include/geek.h``; ``_lib`` is its ctypes
binding and ``api`` the torch-facing wrappers.
"""

from ._lib import GeekError, version  # noqa: F401
