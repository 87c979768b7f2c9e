"""Seeded synthetic inputs for the level-set grain-growth step.

This package only draws random numbers and builds label fields (which grain
owns each voxel of the periodic grid).  It holds none of the method's
arithmetic: both the CPU oracle and the GPU library consume its outputs.
"""
from .labels import (  # noqa: F401
    power_labels,
    compact_labels,
    uniform_voronoi,
    rsa_power_diagram,
    ball_labels,
    slab_labels,
    shoemake_quaternions,
    random_unit_vectors,
    magnetic_energy_density,
)
from .configs import CONFIGS, make_config, config_dt  # noqa: F401
