"""MI355X (gfx950) randomized T-HOSVD / ST-HOSVD with adaptive shifted power iteration.

The method runs in libtucker.so (HIP kernels behind the C ABI declared in
include/tucker.h). This package is its Python binding; the binding is loaded
on first use of any public name, and raises ImportError if the library has
not been built (python -m paper_2506_04840_amd.build).
"""
_PUBLIC = ("rsthosvd", "rthosvd", "sketch", "shifted_power", "orth", "core", "fill_gaussian", "norm2", "Solver",
           "read_info", "workspace_bytes", "op_workspace_bytes", "TuckerError")


def __getattr__(name):
    if name in _PUBLIC:
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
