"""gg_autotune: the chosen launch schedule comes from the candidate set and
every candidate's device time per grain voxel is reported; the steps it takes
(each candidate schedule in turn) give exactly the states of untuned steps, in
both precisions and with both re-initialization schemes: the schedule (launch
order of the grains, the Euclidean variant's work-item tilings) never changes a
value of the functions."""
import numpy as np
import pytest

from synth import make_config
from test_gpu_io import _same

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,redistance", [("fp64", "taxicab"), ("fp32", "taxicab"), ("fp32", "euclid")])
def test_autotune_keeps_results(precision, redistance):
    import paper_1701_06658_amd as gg
    c = make_config(2, N=64, G=125)
    a = gg.Simulation(c["labels"], c["W"], G=c["G"], precision=precision, redistance=redistance)
    b = gg.Simulation(c["labels"], c["W"], G=c["G"], precision=precision, redistance=redistance)
    chosen = a.autotune(c["dt"], 1)
    cands = chosen["candidates"]
    assert len(cands) >= 2 and all(x["ns_per_gv"] > 0 for x in cands)
    picked = (chosen["order_size"], chosen["lds_bytes"], chosen["small_bytes"])
    assert picked in {(x["order_size"], x["lds_bytes"], x["small_bytes"]) for x in cands}
    best = min(cands, key=lambda x: x["ns_per_gv"])
    assert picked == (best["order_size"], best["lds_bytes"], best["small_bytes"])
    n = a.stats()["steps"]
    assert n == len(cands)
    b.step(c["dt"], n)
    _same(a.state(), b.state())
    a.step(c["dt"], 2)
    b.step(c["dt"], 2)
    _same(a.state(), b.state())
    assert np.array_equal(a.volumes(), b.volumes())
