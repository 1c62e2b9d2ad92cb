"""MI355X exponential-integrator library for the Fisher-Kolmogorov glioma model.

The compute lives in ``libexpint.so`` (hand-written HIP kernels for gfx950
behind the C ABI of ``include/expint.h``); this package is its Python binding.
"""

from ._native import ExpIntError, lib  # noqa: F401


def __getattr__(name):
    # torch is imported only when the binding classes are used
    if name in ("ExpInt", "Plan"):
        from . import expint as _e

        return getattr(_e, name)
    raise AttributeError(name)
