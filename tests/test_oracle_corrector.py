"""Pins of the oracle's corrector and labels (sec. 2.1.5):

* an exact +-SDF pair: with psi_1 = -psi_0 the corrector returns psi_0 itself,
  (psi - (-psi)) / 2 = psi, bit for bit (the convolution of -f is -conv(f));
* ties go to the lowest id, in the labels and in the ID-field: two grains with
  identical functions never give the larger id.
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
