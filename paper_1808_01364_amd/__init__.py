"""MI355X-native recursively preconditioned hierarchical interpolative factorization.

The product is librhif.so (HIP for gfx950, C ABI in include/rhif.h); ``rhif`` is its
Python binding. Importing the package does not load the library; the first call does,
and fails loudly if it has not been built.
"""
__all__ = ["rhif"]
