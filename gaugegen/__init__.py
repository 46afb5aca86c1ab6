"""Seeded synthetic inputs: SU(3) link fields, su(3) momenta and gauge transforms.

Used by both the GPU path's tests/benchmark and the CPU oracle's tests. It holds none
of the method's arithmetic (no loops, staples, action, force or exponential map of
the update); exponentials of random algebra elements are taken through ``eigh``.

All fields are numpy complex128 in the canonical layout ``(Lt, Lz, Ly, Lx, 4, 3, 3)``
(site ``((t*Lz + z)*Ly + y)*Lx + x``, direction mu = 0..3 for x, y, z, t), and lattice
dimensions are given as ``L = (Lx, Ly, Lz, Lt)``. Random numbers come from
``numpy.random.default_rng(seed)`` (PCG64).
"""
from .fields import (  # noqa: F401
    generators,
    haar_su3,
    haar_links,
    near_thermal_links,
    near_thermal_links_device,
    momenta,
    gauge_transform,
    unit_links,
    abelian_flux_links,
    field_shape,
    CONFIGS,
    batch_recipe,
    make_config,
    U0,
    BETA,
)
