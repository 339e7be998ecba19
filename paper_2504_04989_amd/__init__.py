"""MI355X-native randomized block Krylov truncated T-SVD (arXiv:2504.04989).

The compute path is the C-ABI library ``libtsvd_rbk.so`` (hand-written HIP
kernels for gfx950) built from ``csrc/``; ``api`` is a thin ctypes binding over
it.  Importing this package does not load the library: ``api`` does, and fails
loudly if it has not been built.
"""
__all__ = ["api", "inputs"]
