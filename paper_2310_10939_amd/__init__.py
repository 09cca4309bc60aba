"""MI355X (gfx950) implementation of the hot path of FastSpectralCluster.

The kernels and the C ABI live in libfsc.so (built from csrc/ by build.py);
`paper_2310_10939_amd.fsc` is the Python binding.  The binding is imported
lazily so that building the library does not need it to exist yet.
"""
import importlib

__all__ = ["fsc", "build"]


def __getattr__(name):
    if name in ("fsc", "build"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
