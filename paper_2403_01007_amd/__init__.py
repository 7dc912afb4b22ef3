"""SCCSD(E) gradients and nonadiabatic couplings on AMD Instinct MI355X.

Thin ctypes binding of libscc.so (include/scc.h).  The binding only
marshals arguments: every step of the method runs in the HIP library.
PyTorch supplies device memory and the stream.
"""
from .binding import (SCC_OK, SccError, Context, Dims, Options, Info, load_library, library_path,
                      EXPORTED_SYMBOLS)

__all__ = ["SCC_OK", "SccError", "Context", "Dims", "Options", "Info", "load_library", "library_path",
           "EXPORTED_SYMBOLS"]
