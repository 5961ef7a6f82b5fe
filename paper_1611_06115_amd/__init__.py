"""MI355X-native k-mismatch character-class DNA scan (arXiv 1611.06115).

The scan, batched scan and serving engine run in the HIP library
``libpmscan.so`` (gfx950); ``scan`` and ``server`` are thin ctypes bindings
over its C ABI (``include/pmscan.h``).  ``synth`` generates seeded inputs.

Submodules are imported on first use so that input generation works on a
machine without the built HIP library.
"""
import importlib

__all__ = ["scan", "synth", "server", "tune"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
