"""MI355X (gfx950) implementation of Greedy Frank-Wolfe multiclass graph segmentation
(arXiv 2508.09738): a HIP library behind the C ABI in include/gfw.h and its binding.

Importing the package loads nothing; `paper_2508_09738_amd.gfw.lib()` loads libgfw.so and
raises if it has not been built.
"""
from . import gfw  # noqa: F401
