"""MI355X (gfx950) multidimensional complex-to-complex FFT.

The binding lives in :mod:`paper_2209_15040_amd.binding` and loads
``libwsfft.so``; names are forwarded from here on first use, so building the
library (``python -m paper_2209_15040_amd.build``) works before it exists.
Using any name without the built library raises ImportError: there is no CPU
fallback.
"""
import importlib


def __getattr__(name):
    if name.startswith("__") or name in ("build",):
        raise AttributeError(name)
    binding = importlib.import_module(__name__ + ".binding")
    if name == "binding":
        return binding
    return getattr(binding, name)
