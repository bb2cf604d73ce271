"""MI355X-native associated Legendre / spherical harmonic transform.

Forward and inverse SHT of degree N (2N Gauss-Legendre latitudes x 4N-1
longitudes) with the associated Legendre transform applied either densely
(on-the-fly recurrence) or through the hierarchically partitioned
interpolative-decomposition butterfly factorization of Bremer, Chen & Yang
(arXiv 2004.11346), all in hand-written HIP kernels for gfx950 behind a C-ABI
(``include/sht.h``).  The Python layer only marshals arguments.

Submodules are imported lazily so that ``paper_2004_11346_amd.inputs`` can be
used without loading the native library.
"""
__all__ = ["inputs", "sht"]


def __getattr__(name):
    import importlib
    if name in ("sht", "inputs", "lib", "autograd"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
