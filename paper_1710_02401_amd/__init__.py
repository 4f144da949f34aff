"""MI355X-native Schwarz Waveform Relaxation (SWR) Galerkin solver for the
N-body Schrodinger equation (Lorin, arXiv 1710.02401).

The hot path lives in libswr.so (HIP kernels for gfx950 behind the C ABI of
include/swr.h); `swr.Solver` is the thin Python binding.
"""
from .swr import (  # noqa: F401
    SWR_TDSE, SWR_TISE, SWR_WARM_GIVEN, SWR_WARM_PLAIN, SWR_WARM_ZERO,
    Solver, Mlp, SWRError, load_library, desc_from_config, EXPORTS,
)
