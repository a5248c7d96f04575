"""R3DSP hot path on MI355X: HIP kernels for gfx950 behind a C ABI (libr3d.so)
with a thin ctypes binding. See include/r3d.h for the contract."""
from . import r3d  # noqa: F401
from .r3d import (  # noqa: F401
    Context, R3DFilter, State, Outputs, R3DError, load,
    R3D_FP32, R3D_FP16_MFMA, R3D_FP16X2_MFMA,
)
