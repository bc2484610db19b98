"""MI355X-native multidimensional CLAHE (Stimper et al., 2019).

The compute path is the C-ABI library ``libmclahe.so`` (hand-written HIP for
gfx950, declared in ``include/mclahe.h``); this package is a thin binding.
Submodules:
    _lib   -- ctypes binding of the C ABI (no torch)
    api    -- tensor entry points: enhance, enhance_batched, autotune, metrics,
              gaussian, median (pre-denoising)
    serve  -- continuous-batching request server
    synth  -- seeded synthetic workloads (no method arithmetic)
    build  -- builds libmclahe.so in-tree
"""
__version__ = "0.1.0"


def __getattr__(name):
    # lazy: importing the package must not require the built library
    if name in ("enhance", "enhance_batched", "autotune", "read_workspace", "plan_for", "make_plans",
                "metrics", "gaussian", "median"):
        from . import api
        return getattr(api, name)
    if name in ("Plan", "MclaheError"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
