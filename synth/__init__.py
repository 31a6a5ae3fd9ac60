"""Seeded synthetic lattice instances.

This package only draws and packages inputs (lattice sizes, grid sizes, Gaussian
exponents, centres, charges, quadrature parameters).  It holds none of the
method's arithmetic, so that both the CPU oracle and the GPU library can read the
same instances without sharing any computation.
"""

from .instances import (  # noqa: F401
    CONFIG_NAMES,
    Instance,
    make_instance,
    make_config,
    config_c4_lattices,
    tiny_instance,
)
