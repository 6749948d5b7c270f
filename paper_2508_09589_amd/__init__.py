"""MI355X-native space-time multigrid solver for transient heat conduction
(Alexandersen & Appel, arXiv 2508.09589): HIP kernels for gfx950 behind the C
ABI of include/st_api.h, with a thin PyTorch-facing wrapper.

Importing the package loads nothing; the HIP library is loaded (and required)
when a Problem is created.
"""

__all__ = ["Problem", "STSolve", "STObjective", "STPNorm", "info_dict"]


def __getattr__(name):
    if name in __all__:
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
