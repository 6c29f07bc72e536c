"""MI355X-native implicit FE step (Zeng & Courtecuisse, arXiv 2306.05893).

The compute path is the HIP library ``libfe_mi355x.so`` behind the C ABI of
``include/fe.h``; this package is its thin binding.  Importing the package
does not load the library; ``FEContext`` / ``Simulation`` do, and fail loudly
if it has not been built.
"""
from ._lib import (FE_COROTATIONAL, FE_FACTOR_ASYNC, FE_FACTOR_DETERMINISTIC, FE_HEX8,
                   FE_MOONEY_RIVLIN, FE_NEO_HOOKEAN, FE_PREC_FP64, FE_PREC_MIXED, FE_STVK,
                   FE_TET4, FEError, load)

__all__ = ["FE_COROTATIONAL", "FE_FACTOR_ASYNC", "FE_FACTOR_DETERMINISTIC", "FE_HEX8",
           "FE_MOONEY_RIVLIN", "FE_NEO_HOOKEAN",
           "FE_PREC_FP64", "FE_PREC_MIXED", "FE_STVK", "FE_TET4", "FEError", "load",
           "FEContext", "Simulation", "Params", "StepOptions", "rollout"]


def __getattr__(name):
    if name in ("FEContext", "Simulation", "Params", "StepOptions", "rollout", "RolloutFn"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
