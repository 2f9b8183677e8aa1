"""MI355X-native adaptive BDDC: a C-ABI library (HIP kernels for gfx950) and
its ctypes binding.  See include/bddc.h for the ABI."""
from .binding import BDDC, BddcError, Server, load, LIB_PATH  # noqa: F401
