"""rwtrsv: sparse triangular solve on equation-rewritten DAGs (MI355X / gfx950).

The HIP library librwtrsv.so does all the work (level analysis, equation
rewriting, level-scheduled and sync-free solves, the adjoint); this package
marshals torch tensors into its C ABI.  There is no CPU fallback: using the
API without the built library raises ImportError.
"""
import importlib

from ._lib import RwtError  # noqa: F401

_LAZY = ("api", "autograd")


def __getattr__(name):
    # the torch-facing API is loaded on first use so that importing the
    # package (e.g. to build it) needs neither torch nor a GPU
    if name in _LAZY or name in ("build",):
        return importlib.import_module("." + name, __name__)
    for mod in _LAZY:
        m = importlib.import_module("." + mod, __name__)
        if hasattr(m, name):
            return getattr(m, name)
    raise AttributeError(name)
