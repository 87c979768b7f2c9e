"""Edge cases of the GPU path against the oracle (FP64, |dphi| <= 1e-10):
a single grain filling the periodic grid (no interface), non-cubic grids with
axes that no tile size divides, a non-integer band half width, and the largest
band half width W = 16."""
import numpy as np
import pytest

from oracle import Oracle
from synth import config_dt, power_labels, uniform_voronoi
from test_gpu_parity import _check_fp64

pytestmark = pytest.mark.gpu


def _pair(labels, W, G):
    import paper_1701_06658_amd as gg
    return Oracle(labels, W, G=G), gg.Simulation(labels, W, G=G, precision="fp64")


@pytest.mark.parametrize("shape", [(40, 52), (24, 30, 36)])
def test_single_grain_fills_the_grid(shape):
    labels = np.zeros(shape, np.int32)
    W = 4.0
    o, s = _pair(labels, W, 1)
    n0 = shape[-1]
    for _ in range(3):
        o.step(config_dt(1.5, n0))
        s.step(config_dt(1.5, n0))
    _check_fp64(o, s, W, f"single grain {shape}")
    st = s.state()
    assert st["alive"][0] and np.all(st["phi"][0] == W)
    assert s.volumes()[0] == float(np.prod(shape))
    assert np.all(s.labels() == 0)


@pytest.mark.parametrize("shape,G,W,sigma", [((46, 70), 30, 5.5, 1.5), ((36, 44, 56), 60, 5.5, 1.5)])
def test_non_cubic_grid_and_fractional_band(shape, G, W, sigma):
    rng = np.random.default_rng(23)
    labels = power_labels(shape, uniform_voronoi(shape, G, rng))
    o, s = _pair(labels, W, G)
    dt = config_dt(sigma, shape[0])  # sigma in voxels along x (n[0])
    for step in range(1, 4):
        o.step(dt)
        s.step(dt)
        _check_fp64(o, s, W, f"{shape} W={W} step {step}")
        assert np.array_equal(o.labels(), s.labels())


def test_largest_band():
    shape = (128, 128)
    rng = np.random.default_rng(29)
    labels = power_labels(shape, uniform_voronoi(shape, 12, rng))
    W = 16.0
    o, s = _pair(labels, W, 12)
    dt = config_dt(3.0, 128)
    for step in range(1, 4):
        o.step(dt)
        s.step(dt)
        _check_fp64(o, s, W, f"W=16 step {step}")
