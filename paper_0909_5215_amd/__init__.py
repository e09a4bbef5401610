"""MI355X (gfx950) hot path of hyperdynamics for driven frictional sliding.

The compute lives in libhd.so (HIP kernels behind the C ABI of include/hd.h);
``paper_0909_5215_amd.hd`` is its ctypes binding.  Importing the package does
not load the library; the first call into ``hd`` does, and fails loudly if it
is missing.
"""
from . import hd  # noqa: F401

__all__ = ["hd"]
