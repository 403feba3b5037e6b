"""MI355X-native evaluation and differentiation of sparse polynomial systems
in complex double, double double and quad double arithmetic.

The compute path is a HIP library with a C ABI (``include/polyeval.h``);
``paper_1402_2626_amd.polyeval`` is its Python binding.  The binding is
imported lazily so that the input generator (``synth``) can be used without
loading the library.
"""
import importlib

__all__ = ["synth", "polyeval"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
