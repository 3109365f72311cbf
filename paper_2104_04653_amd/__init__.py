"""MI355X-native Darcy solve of the Multiscale Robin Coupled Method.

The work runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/mrcm.h`` (``libmrcm.so``); ``paper_2104_04653_amd.mrcm`` is its
ctypes binding.  Build with ``python -m paper_2104_04653_amd.build``.
"""
from .mrcm import MRCMSolver, MRCMError, SurrogateNet, load_library, LIB_PATH  # noqa: F401
