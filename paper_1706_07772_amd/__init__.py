"""MI355X-native (gfx950, HIP, FP64) ReaxFF force evaluation.

The compute path is the HIP library libreaxff_hip.so behind the C ABI in
include/reaxff.h; this package holds its sources (csrc/), its build script
and a thin ctypes binding.
"""
from .binding import (BATCH_MAX_ATOMS, NDESC, NTERMS, SCHEDULES, TERM_NAMES, Batch,  # noqa: F401
                      ListBuffers, ReaxFF, ReaxFFError, Surrogate, load_library)
