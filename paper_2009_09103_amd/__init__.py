"""MI355X-native biased neighbor selection (C-SAW, arXiv 2009.09103).

The compute path is the HIP library ``libcsaw.so`` (C-ABI declared in
``include/csaw.h``); ``paper_2009_09103_amd.csaw`` is its thin ctypes binding.
``paper_2009_09103_amd.inputs`` holds the seeded synthetic input generators.
Submodules are imported lazily so that input generation does not load the GPU
runtime.
"""
import importlib

__all__ = ["csaw", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
