"""MI355X (gfx950) gate-sweep library for QCWAVE's Op1/Op2/Op3 (arXiv:1101.1785).

The compute path is libqcw.so (hand-written HIP kernels behind the C ABI in
include/qcw.h); ``paper_1101_1785_amd._lib`` is its ctypes binding.  The binding
is loaded on first attribute access, so ``python -m paper_1101_1785_amd.build``
works before anything is built; once loaded, a missing library is an error.
"""
import importlib

__all__ = ["lib"]


def __getattr__(name):
    if name in ("lib", "_lib"):
        return importlib.import_module("._lib", __name__)
    raise AttributeError(name)
