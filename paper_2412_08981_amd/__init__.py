"""MI355X-native non-nested multilevel smoothed Schwarz preconditioned FGMRES.

The solver lives in the HIP/C++ library libnnms.so (C ABI in
include/nnms.h); the submodule ``nnms`` is its thin ctypes binding and is
loaded on first use (building the library does not need it).
"""
_EXPORTS = ("FP64", "MIXED", "Batch", "Hierarchy", "Mesh", "NNMSError", "System", "device_bytes_in_use",
            "last_error", "solve_batch")


def __getattr__(name):
    if name in _EXPORTS:
        from . import nnms

        return getattr(nnms, name)
    raise AttributeError(name)
