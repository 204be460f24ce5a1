"""MI355X (gfx950) jump-SDE proton dose engine.

The hot path (per-history transport, fixed-point tally, dose conversion and
the gamma judge) is HIP code in ``libsde.so`` behind the C ABI of
``include/sde.h``; ``paper_2511_03115_amd.sde`` is its ctypes binding.
Importing ``sde`` fails if the library is not built.
"""

__all__ = ["sde", "build"]
