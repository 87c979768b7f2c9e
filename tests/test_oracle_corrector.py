"""Pins of the oracle's corrector and labels (sec. 2.1.5):

* an exact +-SDF pair: with psi_1 = -psi_0 the corrector returns psi_0 itself,
  (psi - (-psi)) / 2 = psi, bit for bit (the convolution of -f is -conv(f));
* ties go to the lowest id, in the labels and in the ID-field: two grains with
  identical functions never give the larger id;
* the sampling rule across the periodic boundary: a box that wraps around
  the grid's edge meets the other grain at the right global voxels, checked
  through an explicit global-index map (-W outside a box).
"""
import numpy as np

from oracle import Oracle
from synth import config_dt


def _field(N, dim):
    ax = np.arange(N, dtype=float)
    if dim == 3:
        z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
        return np.clip(0.37 * x - 0.81 * y + 0.46 * z - 3.3 + 5 * np.sin(x / 7.0), -6.0, 6.0)
    y, x = np.meshgrid(ax, ax, indexing="ij")
    return np.clip(0.6 * x - 0.8 * y - 1.7 + 4 * np.sin(y / 5.0), -6.0, 6.0)[None]


def test_corrector_identity_on_an_exact_pair():
    for dim, N in ((2, 40), (3, 28)):
        f = _field(N, dim)
        shape = f.shape
        o = Oracle(np.zeros(shape, np.int32), 6.0, G=2)
        ext = [N, N, N if dim == 3 else 1]
        o.set_grain(0, True, [0, 0, 0], ext, f)
        o.set_grain(1, True, [0, 0, 0], ext, -f)
        o.keep_intermediates(True)
        o.step(config_dt(1.5, N))
        assert np.array_equal(o.psi(1), -o.psi(0))
        assert np.array_equal(o.phic(0), o.psi(0))
        assert np.array_equal(o.phic(1), o.psi(1))


def test_ties_go_to_the_lowest_id():
    N, W = 48, 6.0
    y, x = np.mgrid[0:N, 0:N]
    # grain 0: the matrix; grains 1 and 2: the same disc with the same function
    labels = ((x - 23.5) ** 2 + (y - 24.5) ** 2 < 10.3 ** 2).astype(np.int32)[None]
    o = Oracle(labels, W, G=3)
    alive, lo, ext = o.box(1)
    o.set_grain(2, True, lo, ext, o.phi(1))
    lab = o.labels()[0]
    assert (lab == 1).sum() > 300 and not (lab == 2).any()
    quat = np.tile([1.0, 0.0, 0.0, 0.0], (3, 1))
    o.set_physics(1, quat=quat, theta_c_deg=15.0)   # builds the ID-fields
    io0 = o.iota(0)
    assert (io0 == 1).any() and not (io0 == 2).any()   # 1 and 2 tie for the matrix
    inside = o.phi(1) > 0
    # no tie for the twins themselves: each one's best other inside is the other twin
    assert np.all(o.iota(2)[inside] == 1) and np.all(o.iota(1)[inside] == 2)
    assert np.all(o.iota(2)[~inside] == 0) and np.all(o.iota(1)[~inside] == 0)


def test_corrector_sampling_across_the_periodic_boundary():
    # a partial box that wraps around x and y against a whole-grid grain: the
    # corrector's other-grain maximum, checked voxel by voxel through an
    # explicit global-index map (outside a box a grain reads -W)
    N, W = 40, 5.0
    rng = np.random.default_rng(17)
    o = Oracle(np.zeros((1, N, N), np.int32), W, G=2)
    f0 = rng.uniform(-W, W, size=(1, N, N))
    lo1, ext1 = np.array([N - 6, N - 3, 0]), np.array([18, 16, 1])
    f1 = rng.uniform(-W, W, size=(1, ext1[1], ext1[0]))
    o.set_grain(0, True, [0, 0, 0], [N, N, 1], f0)
    o.set_grain(1, True, lo1, ext1, f1)
    o.keep_intermediates(True)
    o.step(config_dt(1.5, N))
    psi0, psi1 = o.psi(0)[0], o.psi(1)[0]
    c0, c1 = o.phic(0)[0], o.phic(1)[0]
    other = np.full((N, N), -W)                       # grain 1 seen on the global grid
    ys = (np.arange(ext1[1]) + lo1[1]) % N
    xs = (np.arange(ext1[0]) + lo1[0]) % N
    other[np.ix_(ys, xs)] = psi1
    assert np.array_equal(c0, 0.5 * (psi0 - other))
    assert np.array_equal(c1, 0.5 * (psi1 - psi0[np.ix_(ys, xs)]))
