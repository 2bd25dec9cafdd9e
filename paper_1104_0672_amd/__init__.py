"""MI355X-native hybrid Fourier/direct-space convolution on the sphere.

The compute path lives in libarkcos.so (HIP for gfx950, C ABI in
include/arkcos.h); this package only binds it for PyTorch users.
"""
from .arkcos import ArkcosError, Batch, Plan, choose_radius, load_library, truncation_variance  # noqa: F401
from .autograd import ArkcosConv, convolve  # noqa: F401
