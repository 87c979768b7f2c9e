"""FP64 CPU oracle of the level-set grain-growth step (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this package.  It never imports the GPU library and the GPU
library never imports it.
"""
from .oracle import Oracle, build_oracle, load_library, convolve_box, redistance_box, euclid_sweeps, \
    coarse_sample_box, closest_box, \
    misorientation_deg, pair_weight, num_threads, set_num_threads, ORACLE_CFLAGS  # noqa: F401
