"""MI355X-native COLATUS hot path: direct-summation comoving gravity and the
expansion-aware kick-drift-kick step, as a C-ABI HIP library (libcolatus.so)
with a thin Python binding.

``paper_1208_3444_amd.inputs`` (seeded synthetic inputs) imports no native
code; the binding names (``forces``, ``step``, ``run``, ``adjoint`` ...) are
loaded from ``paper_1208_3444_amd.colatus`` on first use, which fails loudly
if the HIP library has not been built.
"""

_SUBMODULES = ("inputs", "colatus", "build")


def __getattr__(name):
    if name.startswith("_") or name in _SUBMODULES:
        raise AttributeError(name)
    from . import colatus as _c
    return getattr(_c, name)
