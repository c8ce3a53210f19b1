"""MI355X-native Rejection-Free Partial Neighbor Search sampler.

The sampler itself is the HIP library ``libpns.so`` (C ABI, ``include/pns.h``);
``binding`` is its thin ctypes binding, loaded on first use.
"""
import importlib

__all__ = ["binding", "inputs"]


def __getattr__(name):
    if name in ("binding", "inputs", "autograd", "autotune"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
