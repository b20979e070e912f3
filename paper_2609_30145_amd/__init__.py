"""MI355X (gfx950) batched stellar-population forward model and logL.

The compute path is the HIP library libsps.so (C ABI in include/sps.h); this
package holds its build script and a thin ctypes binding.  Importing the
binding does not require a GPU; calling it does.
"""
from .sps import (PRECISIONS, Library, Observation, Server, SpsError, forward, lib, logl,  # noqa: F401
                  logl_grad, logl_lines_joint, logl_static)

__all__ = ["Library", "Observation", "Server", "SpsError", "forward", "logl", "logl_grad", "logl_lines_joint",
           "logl_static", "lib", "PRECISIONS"]
