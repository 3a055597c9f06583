"""MI355X-native local spline simulator (LOSS) of arXiv 2301.05127.

The compute path is the HIP library ``libloss.so`` behind the C ABI in
``include/loss.h``; :mod:`paper_2301_05127_amd.loss` is its ctypes binding.  Importing
this package loads nothing: the binding loads the library on first use and raises if
it is missing.
"""

__all__ = ["inputs", "loss"]
