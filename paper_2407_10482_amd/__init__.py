"""MI355X-native NGP-RT render path: HIP kernels for gfx950 behind a C ABI
(libngprt.so, declared in include/ngprt.h) and a thin PyTorch binding."""
from ._lib import BF16, F32, FP8E4M3, ROI_BOX, ROI_CONTRACT, NgprtError, load_library

__all__ = ["BF16", "F32", "FP8E4M3", "ROI_BOX", "ROI_CONTRACT", "NgprtError", "load_library",
           "Renderer"]


def __getattr__(name):
    if name == "Renderer":
        from .renderer import Renderer
        return Renderer
    raise AttributeError(name)
