"""Argument errors on a live simulation (GPU, through the C ABI): each call is
refused with GG_E_ARG (or GG_E_SMALLBUF) and leaves the state unchanged, so the
simulation keeps stepping exactly as one that never saw the bad call.  Among
them: a state with a non-finite value and one whose box breaks the box rule."""
import ctypes as C

import numpy as np
import pytest

from synth import config_dt, make_config
from test_gpu_io import _same

pytestmark = pytest.mark.gpu


def test_refused_calls_change_nothing():
    import paper_1701_06658_amd as gg
    c = make_config(1)
    a = gg.Simulation(c["labels"], c["W"], G=c["G"], precision="fp64")
    b = gg.Simulation(c["labels"], c["W"], G=c["G"], precision="fp64")
    a.step(c["dt"], 2)
    b.step(c["dt"], 2)
    st = a.state()
    k0 = int(np.nonzero(st["alive"])[0][0])
    phis_nan = [None if p is None else p.copy() for p in st["phi"]]
    phis_nan[k0].flat[0] = np.nan                     # a non-finite value
    ext_bad = st["ext"].copy()
    ext_bad[k0, 0] = c["N"] - 1                       # longer than n - 2P, not the whole axis
    bad = [
        lambda: a.load_state(st["alive"], st["lo"], st["ext"], phis_nan),
        lambda: a.load_state(st["alive"], st["lo"], ext_bad, st["phi"]),
        lambda: a.step(config_dt(20.0, c["N"])),      # kernel radius beyond 2P
        lambda: a.step(-1.0),
        lambda: a.step(float("nan")),
        lambda: a.coarsen((c["N"] * 2, c["N"] * 2, 1)),  # finer, not coarser
        lambda: a.coarsen((40, 30, 1)),                # ratios differ between the axes
        lambda: a.coarsen((20, 20, 1)),                # below 4P + 2
        lambda: a.coarsen((32, 32, 2)),                # 2D needs n[2] == 1
        lambda: a.autotune(c["dt"], 0),
        lambda: a.grain_sdf(c["G"]),
    ]
    for f in bad:
        with pytest.raises(gg.GGError, match="GG_E_ARG"):
            f()
    lo = np.zeros(3, np.int32)
    ext = np.zeros(3, np.int32)
    small = np.zeros(1, np.float64)
    st = a._lib.gg_grain_sdf(a._h, 0, lo.ctypes.data_as(C.c_void_p), ext.ctypes.data_as(C.c_void_p),
                             small.ctypes.data_as(C.c_void_p), 1)
    assert st == 5                                     # GG_E_SMALLBUF, box reported
    assert ext.prod() > 1
    _same(a.state(), b.state())
    a.step(c["dt"], 3)
    b.step(c["dt"], 3)
    _same(a.state(), b.state())
    assert np.array_equal(a.volumes(), b.volumes())
