"""Run-to-run determinism on the GPU: two simulations of the same input, one
on the library's own stream and one on a caller's stream, stepped alternately,
end bit-identical (functions, boxes, ID-fields, volumes, labels).  The step has
no floating-point atomics: reductions run in a fixed order, and the only
atomics (box bounds, occupancy bits, list cursors) give the same result in any
order, so a race or an order dependence would show up here."""
import ctypes as C

import numpy as np
import pytest

from synth import make_config

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,redistance,physics", [("fp32", "taxicab", 0), ("fp32", "euclid", 0),
                                                          ("fp64", "taxicab", 1)])
def test_two_runs_are_bit_identical(precision, redistance, physics):
    import paper_1701_06658_amd as gg
    hip = C.CDLL("libamdhip64.so")
    hip.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
    stream = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(stream)) == 0
    c = make_config(3, N=96, G=400)
    kw = dict(G=c["G"], precision=precision, redistance=redistance)
    if physics:
        rng = np.random.default_rng(9)
        q = rng.normal(size=(c["G"], 4))
        kw.update(physics=gg.PHYS_MISORIENTATION, quat=q / np.linalg.norm(q, axis=1, keepdims=True),
                  theta_c_deg=15.0)
    a = gg.Simulation(c["labels"], c["W"], **kw)
    b = gg.Simulation(c["labels"], c["W"], stream=stream.value, **kw)
    for _ in range(8):
        a.step(c["dt"])
        b.step(c["dt"])
    ba, va = a.values()
    bb, vb = b.values()
    for key in ("lo", "ext", "alive", "offset"):
        assert np.array_equal(ba[key], bb[key]), key
    assert np.array_equal(va, vb)
    if physics:
        assert np.array_equal(a.iota()[1], b.iota()[1])
    assert np.array_equal(a.volumes(), b.volumes())
    assert np.array_equal(a.labels(), b.labels())
    print(f"[{precision} {redistance} physics={physics}] {va.size} values identical, alive {a.alive_count()}",
          flush=True)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_predictor_output_is_bit_identical(precision):
    # the predictor's output of every step, box values far from any interface
    # included (where a wrong value changes no function but may name another
    # neighbour in the ID-field): equal between two runs, step by step
    import paper_1701_06658_amd as gg
    c = make_config(3, N=96, G=400)
    a = gg.Simulation(c["labels"], c["W"], G=c["G"], precision=precision)
    b = gg.Simulation(c["labels"], c["W"], G=c["G"], precision=precision)
    a.keep_intermediates(True)
    b.keep_intermediates(True)
    for step in range(1, 5):
        a.step(c["dt"])
        b.step(c["dt"])
        pa, pb = a.intermediate(0), b.intermediate(0)
        for k in range(c["G"]):
            assert pa["alive"][k] == pb["alive"][k]
            if pa["alive"][k]:
                assert np.array_equal(pa["phi"][k], pb["phi"][k]), (precision, step, k)
                assert np.all(np.abs(pa["phi"][k]) <= c["W"] * (1 + 1e-6)), (precision, step, k)  # sums of taps round
    a.close()
    b.close()
