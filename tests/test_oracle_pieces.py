"""Pins of the oracle's predictor convolution and re-initialization pieces.

Each test checks the oracle against something other than itself: a brute-force
D-dimensional sum, closed-form moments, the exact L1 distance to a plane, or a
brute-force minimum over all reference voxels.
"""
import itertools

import numpy as np
import pytest

from oracle import convolve_box, redistance_box


def _taps(sigma):
    # sampled, truncated, normalised Gaussian (sec. 2.1.4: heat kernel of variance 2t)
    R = int(np.ceil(4 * sigma - 1e-9))
    i = np.arange(-R, R + 1)
    g = np.exp(-(i * i) / (2 * sigma * sigma))
    return R, g / g.sum()


def _sample(f, n, c, fill):
    """Value of a box field (ez, ey, ex) at local coords c=(x, y, z) under the periodic rule."""
    ez, ey, ex = f.shape
    lx, ly, lz = c[0] % n[0], c[1] % n[1], c[2] % n[2]
    if lx >= ex or ly >= ey or lz >= ez:
        return fill
    return f[lz, ly, lx]


@pytest.mark.parametrize("shape,n,sigma", [
    ((5, 7, 9), (16, 16, 16), 1.0),      # interior box, no wrap
    ((5, 7, 9), (9, 16, 5), 0.8),       # ext == n on x and z: full periodic wrap
    ((4, 6, 8), (10, 7, 6), 0.7),       # ext close to n: reads wrap into the box
])
def test_conv_matches_bruteforce_3d(shape, n, sigma):
    rng = np.random.default_rng(1)
    W = 3.0
    f = rng.uniform(-W, W, size=shape)
    out = convolve_box(f, W, sigma, n)
    R, g = _taps(sigma)
    ez, ey, ex = shape
    ref = np.zeros(shape)
    for z, y, x in itertools.product(range(ez), range(ey), range(ex)):
        acc = 0.0
        for (i, gi), (j, gj), (k, gk) in itertools.product(enumerate(g), repeat=3):
            acc += gi * gj * gk * _sample(f, n, (x + i - R, y + j - R, z + k - R), -W)
        ref[z, y, x] = acc
    assert np.max(np.abs(out - ref)) < 1e-13


def test_conv_matches_bruteforce_2d():
    rng = np.random.default_rng(2)
    W, sigma, n = 2.0, 1.2, (12, 9, 1)
    f = rng.uniform(-W, W, size=(1, 9, 7))
    out = convolve_box(f, W, sigma, n)
    R, g = _taps(sigma)
    ref = np.zeros_like(f)
    for y, x in itertools.product(range(9), range(7)):
        acc = 0.0
        for (i, gi), (j, gj) in itertools.product(enumerate(g), repeat=2):
            acc += gi * gj * _sample(f, n, (x + i - R, y + j - R, 0), -W)
        ref[0, y, x] = acc
    assert np.max(np.abs(out - ref)) < 1e-13


def test_conv_preserves_constant_on_full_periodic_box():
    n = (20, 18, 16)
    f = np.full((16, 18, 20), 2.75)
    out = convolve_box(f, 8.0, 2.0, n)
    assert np.max(np.abs(out - 2.75)) < 1e-13


@pytest.mark.parametrize("sigma", [1.0, 1.5, 2.0])
def test_conv_linear_exact_and_second_moment(sigma):
    # symmetric normalised taps keep a linear field and add sigma^2 to x^2
    # (checked away from the box edges, where the -W fill is not reached)
    x = np.arange(64.0)
    R = int(np.ceil(4 * sigma - 1e-9))
    f = np.repeat((0.37 * x - 3.0)[None, :], 64, axis=0)[None]
    out = convolve_box(f, 100.0, sigma, (64, 64, 1))
    core = (0, slice(R, 64 - R), slice(R, 64 - R))
    assert np.max(np.abs(out[core] - f[core])) < 1e-12
    q = np.repeat(((x - 32.0) ** 2)[None, :], 64, axis=0)[None]
    m2 = convolve_box(q, 1e6, sigma, (64, 64, 1))[0, 32, 32]
    # sampled Gaussian truncated at 4 sigma: second moment within 0.2% of sigma^2
    assert abs(m2 - sigma ** 2) < 2e-3 * sigma ** 2


def _plane_field(shape, normal, c, W):
    ez, ey, ex = shape
    z, y, x = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
    nv = np.asarray(normal, float)
    proj = nv[0] * x + nv[1] * y + (nv[2] * z if len(nv) == 3 else 0.0)
    d = (proj - c) / np.max(np.abs(nv))
    return np.clip(d, -W, W)


@pytest.mark.parametrize("seed", range(6))
def test_redistance_planar_is_exact_l1_distance(seed):
    # sec. 2.1.6: exact reference values, taxicab spreading -> the exact L1
    # (taxicab) distance |n.x - c| / ||n||_inf of any plane at every band voxel
    rng = np.random.default_rng(100 + seed)
    W = 6.0
    shape = (26, 26, 26)
    nv = rng.normal(size=3)
    c = float(nv @ np.array([12.6, 13.1, 12.9])) + rng.uniform(-0.5, 0.5)
    phi0 = _plane_field(shape, nv, c, W)
    out = redistance_box(phi0, W, (64, 64, 64))
    m = int(np.ceil(W)) + 1
    core = (slice(m, -m),) * 3
    assert np.max(np.abs(out[core] - phi0[core])) < 1e-12


def test_redistance_planar_2d_exact():
    W = 5.0
    rng = np.random.default_rng(7)
    for _ in range(4):
        nv = rng.normal(size=2)
        c = float(nv @ np.array([15.3, 14.7]))
        phi0 = _plane_field((1, 30, 30), nv, c, W)
        out = redistance_box(phi0, W, (64, 64, 1))
        core = (slice(None), slice(7, -7), slice(7, -7))
        assert np.max(np.abs(out[core] - phi0[core])) < 1e-12


def _ref_values(f, n, W):
    """Reference distances at voxels next to a sign change (written out directly)."""
    ez, ey, ex = f.shape
    dim = 2 if n[2] == 1 else 3
    ref = np.full(f.shape, np.inf)
    for z, y, x in itertools.product(range(ez), range(ey), range(ex)):
        fx = f[z, y, x]
        for a in range(dim):
            for s in (-1, 1):
                c = [x, y, z]
                c[a] += s
                fn = _sample(f, n, c, -W)
                if (fn > 0) != (fx > 0):
                    ref[z, y, x] = min(ref[z, y, x], fx / (fx - fn))
    return ref


@pytest.mark.parametrize("shape,n", [((5, 6, 7), (32, 32, 32)), ((1, 9, 11), (32, 32, 1)),
                                     ((4, 5, 6), (6, 40, 4))])
def test_redistance_matches_bruteforce_min(shape, n):
    rng = np.random.default_rng(11)
    W = 3.0
    f = rng.uniform(-1.0, 1.0, size=shape)
    f[f == 0] = 0.1
    out = redistance_box(f, W, n)
    ref = _ref_values(f, n, W)
    ez, ey, ex = shape
    pts = [(z, y, x) for z, y, x in itertools.product(range(ez), range(ey), range(ex))
           if np.isfinite(ref[z, y, x])]
    brute = np.empty(shape)
    for z, y, x in itertools.product(range(ez), range(ey), range(ex)):
        best = np.inf
        for (pz, py, px) in pts:
            # L1 distance within the box; an axis with ext == n is periodic
            d = 0
            for a, (u, v, e, N) in enumerate(((x, px, ex, n[0]), (y, py, ey, n[1]), (z, pz, ez, n[2]))):
                dd = abs(u - v)
                if e == N:
                    dd = min(dd, N - dd)
                d += dd
            best = min(best, ref[pz, py, px] + d)
        dist = min(best, W)
        brute[z, y, x] = dist if f[z, y, x] > 0 else -dist
    assert np.max(np.abs(out - brute)) < 1e-12
    assert np.all((out > 0) == (f > 0))
    assert np.all(np.abs(out) <= W)
