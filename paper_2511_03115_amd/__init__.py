"""MI355X (gfx950) jump-SDE proton dose engine.

The hot path (per-history transport, fixed-point tally, dose conversion and
the gamma judge) is HIP code in ``libsde.so`` behind the C ABI of
``include/sde.h``; the learned denoiser's kernels sit in the same library
behind ``include/sde_nn.h``.

* ``sde``: ctypes binding of the transport, plans and gamma (import fails if
  the library is not built: there is no CPU fallback);
* ``nn``: ctypes binding of the denoiser network and its single layers;
* ``denoiser``: training on SDE-generated pairs, checkpoints, inference;
* ``judge``: the plain SDE as judge and fallback, time to a 95 % gamma dose;
* ``autotune``: launch-configuration tuning for plans;
* ``build``: compiles the library with hipcc for gfx950.
"""

__all__ = ["sde", "nn", "denoiser", "judge", "autotune", "build"]
