"""MI355X (gfx950) sparse-octree gravitational tree-code after Bedorf, Gaburov &
Portegies Zwart (arXiv:1106.1900).

The compute path is the HIP library ``libbh.so`` (C ABI in ``include/bh.h``);
this package only marshals torch tensors (device memory and the current HIP
stream) into its calls.  There is no CPU fallback: if the library is missing the
import of ``Context`` fails.
"""

from .binding import (  # noqa: F401
    MAC_EQ1,
    MAC_MIN_DIST,
    REQ_DONE,
    REQ_FAILED,
    REQ_QUEUED,
    REQ_RUNNING,
    BHError,
    Cluster,
    Context,
    Server,
    Stats,
    library_path,
    load_library,
    declared_functions,
    forces_static,
    STATIC_MAX_N,
)

__all__ = ["MAC_EQ1", "MAC_MIN_DIST", "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE", "REQ_FAILED", "BHError", "Cluster", "Context", "Server", "Stats", "library_path", "load_library", "declared_functions", "forces_static", "STATIC_MAX_N"]
