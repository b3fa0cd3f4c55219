"""MI355X (gfx950) sketching estimators for full tensor network contraction.

Python binding of libtnsketch.so (C ABI in include/tn_sketch.h).  The binding
only marshals arguments: every step of the estimators runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.

Importing this package requires the built library (see build.py); there is no
fallback path.
"""
from ._binding import *  # noqa: F401,F403  (every public name of the binding)
from ._binding import TNError, NetworkSpec, Plan, MLP, lib_path, load  # noqa: F401
