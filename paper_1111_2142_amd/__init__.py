"""MI355X-native LW-ACM (link-wise artificial compressibility method, arXiv:1111.2142).

The compute path is the HIP library ``liblwacm.so`` (C ABI in
``include/lwacm.h``); ``lwacm`` binds it with ctypes and ``autograd`` wraps
its forward and reverse steps in a ``torch.autograd.Function``.
"""
from . import lwacm  # noqa: F401
from .lwacm import (LWACM_D2Q9, LWACM_D3Q19, LWACM_FP16_DEV, LWACM_FP32, LWACMError,  # noqa: F401
                    Solver, load_library)
