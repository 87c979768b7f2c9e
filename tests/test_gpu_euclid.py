"""Parity of the HIP path's Euclidean re-initialization variant (fast sweeping
with Godunov's upwind update, Jacobi form) with the oracle's, through the C ABI.

Same bars as the method's scheme: FP64 |dphi| <= 1e-10 voxel at every box
voxel after every step, labels identical; FP32 one step from an identical
state within 2e-3 voxel in the band, ownership and volumes as in
test_gpu_parity.py.
"""
import numpy as np
import pytest

from oracle import Oracle
from synth import ball_labels, config_dt, make_config
from test_gpu_parity import _check_fp64, _mixed_one_step, _physics_inputs

pytestmark = pytest.mark.gpu


def _pair(labels, W, G, **kw):
    import paper_1701_06658_amd as gg
    o = Oracle(labels, W, G=G)
    o.set_redistance(1)
    s = gg.Simulation(labels, W, G=G, precision="fp64", redistance="euclid", **kw)
    return o, s


def test_euclid_fp64_trajectory_config1():
    c = make_config(1)
    o, s = _pair(c["labels"], c["W"], c["G"])
    _check_fp64(o, s, c["W"], "euclid cfg1 create")
    for step in range(1, c["steps"] + 1):
        o.step(c["dt"])
        s.step(c["dt"])
        _check_fp64(o, s, c["W"], f"euclid cfg1 step {step}")
        assert np.array_equal(o.labels(), s.labels())


def test_euclid_fp64_3d_voronoi():
    # the 3D uniform Voronoi workload cut to 64^3 and 125 grains
    c = make_config(2, N=64, G=125)
    o, s = _pair(c["labels"], c["W"], c["G"])
    for step in range(1, 4):
        o.step(c["dt"])
        s.step(c["dt"])
        _check_fp64(o, s, c["W"], f"euclid cfg2/64 step {step}")
    assert np.array_equal(o.labels(), s.labels())


@pytest.mark.parametrize("dim,N,R0", [(2, 96, 20.0), (3, 48, 12.0)])
def test_euclid_fp64_ball_with_full_periodic_matrix(dim, N, R0):
    # grain 0's box wraps on every axis: the sweeps read across the seam
    n = (N, N) if dim == 2 else (N, N, N)
    W, sigma = (6.0, 1.5) if dim == 2 else (8.0, 2.0)
    o, s = _pair(ball_labels(n, R0), W, 2)
    dt = config_dt(sigma, N)
    for step in range(8 if dim == 2 else 4):
        o.step(dt)
        s.step(dt)
    _check_fp64(o, s, W, f"euclid ball dim={dim}")


def test_euclid_fp64_with_bulk_term():
    # the ID-field carry and the correction epilogue next to the variant
    labels, gphys, ophys = _physics_inputs("bulk")
    G = int(labels.max()) + 1
    W, sigma = 8.0, 2.0
    o, s = _pair(labels, W, G, **gphys)
    o.set_physics(**ophys)
    dt = config_dt(sigma, labels.shape[0])
    for step in range(1, 3):
        o.step(dt)
        s.step(dt)
        _check_fp64(o, s, W, f"euclid bulk step {step}")


def test_euclid_mixed_one_step_config1():
    c = make_config(1)
    o = Oracle(c["labels"], c["W"], G=c["G"])
    o.set_redistance(1)
    for start in (0, 6):
        _mixed_one_step(o, c["dt"], c["W"], c["G"], f"euclid cfg1 from step {start}", redistance="euclid")
        o.step(c["dt"], 5)


def test_euclid_mixed_one_step_3d():
    c = make_config(2, N=64, G=125)
    o = Oracle(c["labels"], c["W"], G=c["G"])
    o.set_redistance(1)
    o.step(c["dt"])
    _mixed_one_step(o, c["dt"], c["W"], c["G"], "euclid cfg2/64 from step 1", redistance="euclid")
