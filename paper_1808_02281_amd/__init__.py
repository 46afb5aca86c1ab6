"""MI355X (gfx950) implementation of the one-loop Symanzik improved gauge action, its
molecular-dynamics force and a leapfrog update (arXiv:1808.02281, Sec. II).

The computation is in hand-written HIP kernels behind the C ABI of include/sym.h
(libsym.so); this package is a thin binding over torch device memory and streams.
"""
from .api import (  # noqa: F401
    action,
    action_grad,
    batch_autotune,
    force_batch,
    coeffs,
    field_shape,
    force,
    md_leapfrog,
    pack,
    profile_collect,
    profile_enable,
    prec_of,
    release_workspaces,
    set_coeffs_override,
    set_force_algorithm,
    unpack,
    volume,
    workspace,
    workspace_bytes,
)
from .autograd import symanzik_action  # noqa: F401,E402
