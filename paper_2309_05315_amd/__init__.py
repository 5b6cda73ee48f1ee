"""MI355X-native Method of Averaged Marginals (MAM) for Wasserstein barycenters.

The numerical work runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/mam.h`` (library ``libmam.so`` in this package).  The
Python layer only marshals arguments; importing the package does not load the
library, ``paper_2309_05315_amd.mam`` does.
"""
__all__ = ["inputs"]
