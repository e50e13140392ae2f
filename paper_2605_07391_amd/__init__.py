"""MERBIT merge-path SpMV for AMD Instinct MI355X (gfx950).

The compute lives in ``libmerbit.so`` (HIP kernels behind the C ABI of
``include/merbit.h``); ``merbit`` is its thin Python binding.
"""
from .merbit import (EXPORTED, F32, F64, MerbitError, Plan, library_path, load,  # noqa: F401
                     version)

__all__ = ["Plan", "MerbitError", "load", "library_path", "version", "EXPORTED", "F32", "F64"]
