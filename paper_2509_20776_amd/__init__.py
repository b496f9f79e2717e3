"""MI355X (gfx950) sparse-matrix permutation, extraction and assignment.

The compute path is libhipperm.so (hand-written HIP kernels behind the C ABI
in include/hipperm.h); the submodule `hipperm` is its thin Python binding.
Importing the binding fails loudly when the library has not been built;
there is no CPU fallback.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhipperm.so")
