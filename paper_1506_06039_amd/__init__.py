"""MI355X-native translation search of moco (arXiv:1506.06039), section 2.

The compute lives in ``libmoco.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/moco.h``); ``paper_1506_06039_amd.moco`` is its Python binding.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmoco.so")
