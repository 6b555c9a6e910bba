"""Batched, differentiable dense QP solver for AMD MI355X (gfx950).

Hot path: the primal-dual interior point forward solve of many small QPs and the
backward pass that reuses the final factorization (Amos & Kolter 2017, OptNet,
Section 3).  All arithmetic runs in the HIP library ``libqpmi.so`` behind the C
ABI declared in ``include/qpmi.h``; the Python modules only marshal arguments.

Submodules are imported lazily so that ``synth`` (input generators) works on
hosts without a GPU.
"""
import importlib

__all__ = ["binding", "function", "synth", "varlen", "serve", "autotune"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
