"""FP64 CPU oracle for the one-loop Symanzik gauge action and force (arXiv:1808.02281, Sec. II)
for the asqtad / HISQ fat-link smearing and its path force (Secs. "Asqtad fermion",
"HISQ fermion"), and for the Wilson-clover fermion matrix and its force at fixed X, Y
(Sec. "Wilson fermion action with clover term").

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package. It shares no code with the GPU library
(``paper_1808_02281_amd``) and neither imports the other.

Pinned by ``tests/test_oracle_*.py`` against closed forms, exact symmetries, a numpy
brute-force enumeration, finite differences of the action and leapfrog invariants.
"""
from .oracle import (  # noqa: F401
    coeffs,
    loop_table,
    action,
    force,
    force_links,
    staple_sums,
    local_action,
    su3_exp,
    kinetic,
    leapfrog,
    num_threads,
    set_num_threads,
    FAT_CLASSES,
    fat_paths,
    fat_links,
    fat_links_links,
    fat_grad,
    fat_grad_links,
    fat_force_from_grad,
    gamma,
    clover_leaves,
    wilson_apply,
    wilson_psi,
    wilson_force,
    wilson_force_links,
    gell_mann,
    lie_derivative,
)
