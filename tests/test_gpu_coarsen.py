"""Parity of the HIP path's grid coarsening (gg_coarsen) with the oracle's,
through the C ABI: FP64 bit-identical to 1e-10 voxel right after coarsening and
after the steps that follow on the coarser grid (labels identical), at integer
and non-integer ratios, with whole-axis boxes and with the bulk term; FP32 from
the identical oracle state within the mixed bars of test_gpu_parity.py.
"""
import numpy as np
import pytest

from oracle import Oracle
from synth import ball_labels, config_dt, make_config
from test_gpu_parity import TOL_MIXED, _check_fp64, _physics_inputs
from _compare import compare_states

pytestmark = pytest.mark.gpu


def _pair(labels, W, G, precision="fp64", **kw):
    import paper_1701_06658_amd as gg
    return Oracle(labels, W, G=G), gg.Simulation(labels, W, G=G, precision=precision, **kw)


def test_coarsen_fp64_config1_then_steps():
    c = make_config(1)
    o, s = _pair(c["labels"], c["W"], c["G"])
    o.step(c["dt"], 3)
    s.step(c["dt"], 3)
    o.coarsen((32, 32, 1))
    s.coarsen((32, 32, 1))
    _check_fp64(o, s, c["W"], "cfg1 coarsened to 32^2")
    assert np.array_equal(o.labels(), s.labels())
    dt = config_dt(c["sigma"], 32)
    for step in range(1, 5):
        o.step(dt)
        s.step(dt)
        _check_fp64(o, s, c["W"], f"cfg1/32 step {step}")
        assert np.array_equal(o.labels(), s.labels())


@pytest.mark.parametrize("Np", [36, 54])
def test_coarsen_fp64_3d_voronoi(Np):
    # ratio 2 and 4/3 from a 72^3 / 80-grain cut of the 3D Voronoi workload
    c = make_config(2, N=72, G=80)
    o, s = _pair(c["labels"], c["W"], c["G"])
    o.step(c["dt"], 2)
    s.step(c["dt"], 2)
    o.coarsen((Np, Np, Np))
    s.coarsen((Np, Np, Np))
    _check_fp64(o, s, c["W"], f"cfg2/72 coarsened to {Np}^3")
    dt = config_dt(c["sigma"], Np)
    for step in range(1, 3):
        o.step(dt)
        s.step(dt)
        _check_fp64(o, s, c["W"], f"cfg2/72->{Np} step {step}")
    assert np.array_equal(o.labels(), s.labels())


def test_coarsen_fp64_whole_axis_boxes():
    # a sphere in a matrix grain whose box is the whole periodic grid
    o, s = _pair(ball_labels((64, 64, 64), 14.0), 8.0, 2)
    o.coarsen((48, 48, 48))
    s.coarsen((48, 48, 48))
    _check_fp64(o, s, 8.0, "ball 64 -> 48")
    dt = config_dt(2.0, 48)
    o.step(dt, 2)
    s.step(dt, 2)
    _check_fp64(o, s, 8.0, "ball 48 after 2 steps")


def test_coarsen_fp64_bulk_term():
    labels, gphys, ophys = _physics_inputs("bulk")
    G = int(labels.max()) + 1
    o, s = _pair(labels, 8.0, G, **gphys)
    o.set_physics(**ophys)
    dt = config_dt(2.0, 64)
    o.step(dt)
    s.step(dt)
    o.coarsen((48, 48, 48))
    s.coarsen((48, 48, 48))
    _check_fp64(o, s, 8.0, "bulk 64 -> 48")
    dt = config_dt(2.0, 48)
    for step in range(1, 3):
        o.step(dt)
        s.step(dt)
        _check_fp64(o, s, 8.0, f"bulk 48 step {step}")


def test_coarsen_mixed_from_oracle_state():
    import paper_1701_06658_amd as gg
    c = make_config(2, N=72, G=80)
    o = Oracle(c["labels"], c["W"], G=c["G"])
    o.step(c["dt"], 2)
    st = o.state()
    s = gg.Simulation(o.labels(), c["W"], G=c["G"], precision="fp32")
    s.load_state(st["alive"], st["lo"], st["ext"], st["phi"])
    o.coarsen((36, 36, 36))
    s.coarsen((36, 36, 36))
    a, b = o.state(), s.state()
    r = compare_states(a, b, o.n, c["W"], band_only=True)
    print(f"[mixed coarsen] max|dphi| (band) = {r['max_abs']:.3e} alive_mismatch={r['alive_mismatch']}", flush=True)
    assert r["alive_mismatch"] == 0 and r["box_mismatch"] == 0
    assert r["max_abs"] <= TOL_MIXED
    vo, vg = o.volumes(), s.volumes()
    big = vo >= 50
    assert np.all(np.abs(vg[big] - vo[big]) <= 5e-3 * vo[big])
