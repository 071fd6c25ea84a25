"""MI355X hybrid symplectic step (Mercury+ integrator of Mercury-Arxes) -- Python binding.

A thin ctypes layer over ``libmx.so`` (include/mx.h).  It marshals torch tensors
(device memory) and a torch stream; every step of the method runs in the HIP
kernels of the library.  There is no CPU fallback: if the library is missing the
import of any entry point raises.
"""
from ._binding import (  # noqa: F401
    Adjoint,
    Batch,
    MxError,
    Params,
    System,
    flag_pairs,
    gas_drag,
    gravity,
    hybrid_run,
    kepler_drift,
    lib,
    lib_path,
    make_params,
)
