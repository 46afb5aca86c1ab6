"""MI355X (gfx950) implementation of the one-loop Symanzik improved gauge action, its
molecular-dynamics force and a leapfrog update (arXiv:1808.02281, Sec. II), and of the
asqtad/HISQ fat-link smearing with its path force (Secs. "Asqtad fermion", "HISQ fermion"),
and the Wilson-clover fermion force for given vectors X, Y (Sec. "Wilson fermion action
with clover term").

The computation is in hand-written HIP kernels behind the C ABI of include/sym.h
(libsym.so); this package is a thin binding over torch device memory and streams.
"""
from .api import (  # noqa: F401
    action,
    action_grad,
    batch_autotune,
    force_batch,
    check_links,
    coeffs,
    fat_force,
    fat_links,
    fat_workspace,
    field_shape,
    force,
    md_leapfrog,
    new_fat_workspace,
    pack,
    pack_spinor,
    profile_collect,
    profile_enable,
    prec_of,
    release_workspaces,
    reunitarise,
    set_coeffs_override,
    set_force_algorithm,
    unpack,
    unpack_spinor,
    spinor_shape,
    wilson_force,
    wilson_workspace,
    volume,
    workspace,
    workspace_bytes,
)
from .autograd import fat_smear, symanzik_action  # noqa: F401,E402
