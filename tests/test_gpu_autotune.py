"""gg_autotune: the chosen LDS budgets come from the candidate set, and the
steps it takes (each candidate tiling in turn) give exactly the states of
untuned steps, in both precisions: the work-item tiling changes the schedule,
never a value of the functions (grain volumes, sums of per-work-item partial
sums, agree to rounding)."""
import numpy as np
import pytest

from synth import make_config
from test_gpu_io import _same

pytestmark = pytest.mark.gpu

CANDIDATES = {(40960, 26624), (32768, 20480), (40960, 20480), (40960, 32768), (49152, 26624), (49152, 32768),
              (32768, 26624)}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_keeps_results(precision):
    import paper_1701_06658_amd as gg
    c = make_config(2, N=64, G=125)
    a = gg.Simulation(c["labels"], c["W"], G=c["G"], precision=precision)
    b = gg.Simulation(c["labels"], c["W"], G=c["G"], precision=precision)
    chosen = a.autotune(c["dt"], 1)
    assert chosen in CANDIDATES
    n = a.stats()["steps"]
    assert n == len(CANDIDATES)
    b.step(c["dt"], n)
    _same(a.state(), b.state())
    a.step(c["dt"], 2)
    b.step(c["dt"], 2)
    _same(a.state(), b.state())
    # volumes are sums of per-work-item partial sums: equal to rounding
    assert np.allclose(a.volumes(), b.volumes(), rtol=1e-12, atol=0)
