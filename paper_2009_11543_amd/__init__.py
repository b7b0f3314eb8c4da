"""Compressed key sort (Kwon et al., arXiv 2009.11543) for AMD MI355X.

The native library ``libckey.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/ckey.h``) does all the work; ``paper_2009_11543_amd.ckey``
is its thin Python binding and fails loudly if the library is not built.
``paper_2009_11543_amd.datagen`` holds the seeded synthetic key generators.
"""
import importlib

__all__ = ["ckey", "datagen"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
