"""MI355X (gfx950) sign function of triangular matrices.

``signtri`` is the Python binding of ``libsigntri.so`` (C ABI in
``include/signtri.h``); ``workloads`` draws the seeded synthetic inputs.
"""
from . import workloads  # noqa: F401
from .signtri import (  # noqa: F401
    SignTriError,
    plan_host,
    release,
    sign_general_batched,
    sign_tri,
    sign_tri_batched,
    strerror,
    workspace_size,
)
