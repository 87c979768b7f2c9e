"""Edge cases of the GPU path against the oracle (FP64, |dphi| <= 1e-10):
a single grain filling the periodic grid (no interface), non-cubic grids with
axes that no tile size divides, a non-integer band half width, the largest
band half width W = 16, and twin grains (identical functions) whose ties go
to the lowest id."""
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


def test_twin_grains_tie_to_the_lowest_id():
    # two grains with identical functions on the same box: labels and ID-fields
    # take the lower id, and the corrector sees each twin's best other as the
    # other twin: a zero corrected function inside, so both twins vanish in the
    # first step and the matrix takes their voxels, on both sides alike
    import paper_1701_06658_amd as gg
    N, W, G = 48, 6.0, 3
    y, x = np.mgrid[0:N, 0:N]
    labels = ((x - 23.5) ** 2 + (y - 24.5) ** 2 < 10.3 ** 2).astype(np.int32)[None]
    h = np.radians(20.0) / 2.0
    quat = np.array([[1.0, 0.0, 0.0, 0.0], [np.cos(h), 0.0, 0.0, np.sin(h)],
                     [np.cos(h), 0.0, 0.0, np.sin(h)]])
    o = Oracle(labels, W, G=G)
    alive, lo, ext = o.box(1)
    o.set_grain(2, True, lo, ext, o.phi(1))
    o.set_physics(1, quat=quat, theta_c_deg=15.0)
    st = o.state()
    s = gg.Simulation(labels, W, G=G, precision="fp64", physics=gg.PHYS_MISORIENTATION, quat=quat,
                      theta_c_deg=15.0)
    s.load_state(st["alive"], st["lo"], st["ext"], st["phi"],
                 [o.iota(k) if st["alive"][k] else None for k in range(G)])
    lab = s.labels()
    assert np.array_equal(lab, o.labels()) and (lab == 1).any() and not (lab == 2).any()
    for step in range(1, 3):
        o.step(config_dt(1.5, N))
        s.step(config_dt(1.5, N))
        _check_fp64(o, s, W, f"twins step {step}")
        assert np.array_equal(s.labels(), o.labels())
        assert s.alive_count() == o.alive_count() == 1
        _, io_gpu = s.iota()
        io_orc = np.concatenate([o.iota(k).ravel() for k in range(G) if o.box(k)[0]])
        assert np.array_equal(io_gpu, io_orc)
    s.close()


def _max_tile_coverage(st, shape_xyz, tile_xyz):
    """Most boxes that cover one corrector tile (host count from the box table)."""
    nt = [n // t for n, t in zip(shape_xyz, tile_xyz)]
    cover = np.zeros(nt[::-1], np.int32)  # (z, y, x)
    for k in np.nonzero(st["alive"])[0]:
        sets = []
        for a in range(3):
            cells = (st["lo"][k][a] + np.arange(st["ext"][k][a])) % shape_xyz[a]
            sets.append(np.unique(cells // tile_xyz[a]))
        cover[np.ix_(sets[2], sets[1], sets[0])] += 1
    return int(cover.max())


def test_tiles_covered_by_more_than_64_boxes():
    # 300 grains in 32^3 with W = 4: about 100 boxes meet each 16x8x4 corrector
    # tile, so the corrector walks its coverage list in several chunks of 64
    shape = (32, 32, 32)
    rng = np.random.default_rng(37)
    labels = power_labels(shape, uniform_voronoi(shape, 300, rng))
    W = 4.0
    o, s = _pair(labels, W, 300)
    cov = _max_tile_coverage(s.state(), (32, 32, 32), (16, 8, 4))
    print(f"[coverage] most boxes on one tile: {cov}", flush=True)
    assert cov > 64
    dt = config_dt(1.5, 32)
    for step in range(1, 4):
        o.step(dt)
        s.step(dt)
        _check_fp64(o, s, W, f"coverage > 64, step {step}")
        assert np.array_equal(o.labels(), s.labels())
