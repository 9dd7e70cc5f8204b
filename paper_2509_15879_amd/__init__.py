"""MI355X-native θ-scheme solver for the singular parabolic and the
drift-diffusion continuity equations on the unit disk in polar coordinates
(arXiv:2509.15879, Ch. 2 and Ch. 3).

The compute path is the HIP library ``libpolardisk.so`` (C ABI in
``include/polardisk.h``); ``paper_2509_15879_amd.polardisk`` is its ctypes
binding.  Build it with ``python -m paper_2509_15879_amd.build``.
"""

__all__ = ["polardisk", "build"]
