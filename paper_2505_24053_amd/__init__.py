"""MI355X-native exact Gaussian ray renderer (3DGEER, arXiv 2505.24053).

The compute path lives in the HIP library ``libgeer.so`` (C ABI declared in
``include/geer.h``); this package only marshals arguments to it.  Importing
the package does not load the library; the first call does, and fails loudly
when the library has not been built.
"""
__all__ = ["synth"]
