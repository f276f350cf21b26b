"""ORACLE -- test infrastructure, not part of the product.

A plain, slow, FP64 CPU implementation of the sparsified-NetMF hot path,
written from the paper (arXiv 2302.07084): the per-edge downsampled
PathSampling sparsifier (section 5.2 and the two sampling algorithms), the
truncated logarithm of Eq. (1), the fast randomized SVD built on eigSVD
(section 4.2, Algorithms "eigSVD" and "Fast Randomized SVD"), and the
Chebyshev spectral propagation (section 4.3).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never links or calls
it, and this package never imports the GPU library.
"""
from .netmf import *  # noqa: F401,F403
