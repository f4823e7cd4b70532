"""Coherent Fusion pose scoring on AMD Instinct MI355X (gfx950).

The scoring path is a HIP library (libcf.so, C ABI in include/cf.h); `cfabi`
is its thin ctypes binding and `Scorer` a convenience wrapper.  Importing the
package does not load the library; using it does, and fails loudly if it is not
built.
"""
import importlib

__all__ = ["cfabi", "Scorer"]


def __getattr__(name):
    if name == "cfabi":
        return importlib.import_module(".cfabi", __name__)
    if name == "Scorer":
        return importlib.import_module(".scorer", __name__).Scorer
    raise AttributeError(name)
