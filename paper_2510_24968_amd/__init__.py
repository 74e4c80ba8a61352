"""MI355X-native direct-SCF Fock build (McMurchie-Davidson ERIs over
Schwarz-screened shell quartets, digested into J and K on the fly).

The work runs in libfsim.so (HIP kernels for gfx950 behind the C ABI of
include/fsim.h); this package is its thin Python binding."""

from .fsim import (  # noqa: F401
    FSIM_FP64,
    FSIM_MIXED,
    Batch,
    Context,
    FsimError,
    LIBPATH,
    lib,
)
