"""MERBIT merge-path SpMV for AMD Instinct MI355X (gfx950).

The compute lives in ``libmerbit.so`` (HIP kernels behind the C ABI of
``include/merbit.h``); ``merbit`` is its thin Python binding.
"""
from .merbit import (EXPORTED, F32, F64, MerbitError, Plan, column_scale,  # noqa: F401
                     gather_values, library_path, load, tune,
                     version)

__all__ = ["Plan", "MerbitError", "load", "library_path", "tune", "gather_values", "column_scale",
           "version", "EXPORTED", "F32", "F64"]
