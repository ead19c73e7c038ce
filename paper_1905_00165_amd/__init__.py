"""MI355X (gfx950) factorization-based DPP sampler.

The sampler itself is the HIP library libdpp.so (C ABI in include/dpp.h);
`binding` is its thin Python front end and `workloads` builds seeded inputs.
Importing the package loads nothing native; the library is loaded on first
use and its absence is an error.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "binding"]


def __getattr__(name):
    if name == "binding":
        import importlib
        return importlib.import_module(__name__ + ".binding")
    raise AttributeError(name)
