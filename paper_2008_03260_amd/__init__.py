"""MI355X-native SLASH hot path: DOPH hashing, bottom-R reservoir tables,
count-min top-k queries, batched and served forms.

The compute path is ``libslash.so`` (HIP kernels for gfx950, C ABI in
``include/slash.h``); ``paper_2008_03260_amd.api`` is its ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
__all__ = ["api", "build"]
