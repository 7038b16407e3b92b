"""MI355X-native flux-reconstruction residual and Jacobian library.

The compute path lives in ``libfr.so`` (HIP, gfx950) behind a C ABI declared
in ``include/fr.h``; :mod:`paper_2105_08632_amd.fr` is the thin ctypes
binding.  :mod:`paper_2105_08632_amd.inputs` builds seeded synthetic meshes
and states.  Importing the package loads nothing; the library is loaded on
first use and a missing build is an error, never a fallback.
"""
__all__ = ["inputs"]
