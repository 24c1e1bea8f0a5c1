"""MI355X (gfx950) fast multipole method for the 3-D Laplace N-body problem,
after Ltaief & Yokota, "Data-Driven Execution of Fast Multipole Methods".

The compute path is the HIP library libfmm_mi355x.so (C ABI in
include/fmm.h); `fmm` is its Python binding, `autograd` the
torch.autograd.Function around it, `trace` summaries of the device task
trace, `workloads` the seeded input generators.
"""

__all__ = ["Plan", "evaluate", "load_library", "FMMEnergy", "fmm_energy"]


def __getattr__(name):
    if name in ("FMMEnergy", "fmm_energy"):
        from . import autograd as _ag
        return getattr(_ag, name)
    if name in __all__:
        from . import fmm as _fmm
        return getattr(_fmm, name)
    raise AttributeError(name)
