"""MI355X (gfx950) split-step Crank-Nicolson step for the 3D fully anisotropic
Gross-Pitaevskii equation (Vudragovic et al., Comput. Phys. Commun. 183
(2012) 2021).

The computation lives in libgpssc.so (hand-written HIP kernels behind the C
ABI of include/gpssc.h); this package is its Python binding.  The library is
loaded on first use, so importing the package (or its seeded input
generators in ``inputs``) needs no GPU.
"""
from ._binding import (  # noqa: F401
    C64, C64_F64, C128, IMAG, R32, R64, REAL, EXPORTS, KERNELS, Batch, GPError, GPInvalid, GPNoMemory, GPNonFinite,
    Plan, Server,
    footprint_bytes, lib, library_path, request_bytes, step_noalloc, sweep_shape, sweep_tables,
)
