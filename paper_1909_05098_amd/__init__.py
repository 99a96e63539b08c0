"""MI355X (gfx950) FED-FEM bio-heat library: C ABI in libfedfem.so, ctypes
binding in `fedfem`."""
from . import fedfem  # noqa: F401
from .fedfem import (FP32C, FP64, SOURCE_CONSISTENT, SOURCE_NODAL,  # noqa: F401
                     Batch, FedFemError, Handle, load)
