"""MI355X-native GPU Faster Mean Shift (Euclidean), after You et al., arXiv 2112.13891.

The compute path is ``libfms.so`` (hand-written HIP kernels for gfx950 behind a
C ABI, declared in ``include/fms.h``).  This package only loads it and marshals
torch tensors; nothing here computes the method.  Submodules are imported on
first use so that ``paper_2112_13891_amd.workloads`` can be used without the
library.
"""
import importlib

__all__ = ["fit", "step", "assign", "MeanShiftT", "workloads", "MeanShiftError"]


def __getattr__(name):
    if name in ("fit", "step", "assign", "MeanShiftError", "Params", "lib", "seed_draw"):
        return getattr(importlib.import_module(".api", __name__), name)
    if name in ("MeanShiftT",):
        return getattr(importlib.import_module(".autograd", __name__), name)
    if name == "workloads":
        return importlib.import_module(".workloads", __name__)
    raise AttributeError(name)
