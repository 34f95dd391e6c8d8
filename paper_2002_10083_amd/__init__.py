"""MI355X-native Markov-clustering expansion library (arXiv 2002.10083 hot path).

The compute lives in ``libmcl.so`` (HIP kernels for gfx950, C ABI in
``include/mcl.h``); ``paper_2002_10083_amd.mcl`` is its ctypes binding.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmcl.so")


def build() -> str:
    from .build import build as _b
    return _b()
