"""MI355X-native CGKS-5th / GKS-2nd stage sweep (arXiv 2508.19911).

The compute path is the C-ABI library ``libcgks.so`` built from ``csrc/`` (hand-written HIP for
gfx950); :mod:`paper_2508_19911_amd.cgks` is the thin ctypes binding over it.  Importing the package
does not load the library; :func:`paper_2508_19911_amd.cgks.load` does, and fails loudly when the
library is missing.
"""
__all__ = ["inputs", "cgks"]
