"""MI355X (gfx950) level-set grain growth: one timestep of the local level-set
method of Miessen et al. (arXiv:1701.06658) over all grains, in hand-written HIP
kernels behind a C ABI (include/gg.h)."""
from .gg import (GG_FP32, GG_FP64, GG_REDIST_EUCLID, GG_REDIST_TAXICAB, PHYS_BULK,  # noqa: F401
                 PHYS_MISORIENTATION, PHYS_NONE,
                 EXPORTS, GGError, Simulation, load_library, version)
