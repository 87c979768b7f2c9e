"""Pins of the oracle's interface areas and boundary energy (the energy
functional, Eq. Energyfunctional): A_k = sum of |grad H(phi_k)| with the
smoothed Heaviside H = clamp(phi + 1/2, 0, 1) of the volume.

* axis-aligned flat boundaries: exactly the cross-section per boundary (the
  central differences telescope along every line);
* oblique periodic plane arrays: within 4% of the exact area (the clamped ramp's
  central differences overestimate slightly off the axes);
* a smoothed sphere / circle: within 3% / 2.5% of the area of the sphere /
  circle of the same volume; the shrinking sphere's area falls linearly at
  8 pi kappa_s sigma^2 per step (R^2 falls at 2 kappa_s sigma^2);
* a bicrystal with misorientation theta < theta_c: the weighted area is
  gamma(theta) = (theta/theta_c)(1 - ln(theta/theta_c)) times the area;
* curvature flow dissipates energy: the boundary energy of a Voronoi start
  falls at every step.
"""
import numpy as np
import pytest

from oracle import Oracle
from synth import ball_labels, config_dt, make_config
from test_oracle_coarsen import _slab_field
from test_oracle_step import _slab_state


@pytest.mark.parametrize("dim", [2, 3])
def test_axis_aligned_boundaries_exact(dim):
    N = 48
    o = Oracle(np.zeros((1 if dim == 2 else N, N, N), np.int32), 6.0, G=2)
    _slab_state(o, N, 10.25, 30.6, 6.0, dim)
    a, w = o.areas()
    assert np.allclose(a, 2 * N ** (dim - 1), rtol=0, atol=1e-9)
    assert np.array_equal(a, w)


@pytest.mark.parametrize("dim", [2, 3])
def test_oblique_plane_arrays(dim):
    N, W, L = 48, 4.0, 24.0
    d = np.array([0.5, 1.0, 1.0]) if dim == 3 else np.array([0.5, 1.0])
    f = _slab_field(N, d, L, 0.37, dim)
    shape = (N, N, N) if dim == 3 else (1, N, N)
    o = Oracle((f <= 0).astype(np.int32).reshape(shape), W, G=2)
    ext = [N, N, N if dim == 3 else 1]
    o.set_grain(0, True, [0, 0, 0], ext, np.clip(f, -W, W))
    o.set_grain(1, True, [0, 0, 0], ext, np.clip(-f, -W, W))
    a, _ = o.areas()
    # planes d.x = c + k L / 2, (L / 2) / |d| apart: area N^D |d| 2 / L
    exact = N ** dim * np.linalg.norm(d) * 2.0 / L
    assert np.all(np.abs(a / exact - 1.0) < 0.04), a / exact


def test_sphere_and_circle_areas():
    o = Oracle(ball_labels((64, 64, 64), 14.0), 8.0, G=2)
    o.step(config_dt(2.0, 64))
    a, _ = o.areas()
    V = o.volumes()[1]
    assert abs(a[1] / (36.0 * np.pi * V * V) ** (1.0 / 3.0) - 1.0) < 0.03
    o2 = Oracle(ball_labels((96, 96), 20.0), 6.0, G=2)
    o2.step(config_dt(1.5, 96))
    a, _ = o2.areas()
    V = o2.volumes()[1]
    assert abs(a[1] / (2.0 * np.sqrt(np.pi * V)) - 1.0) < 0.025


def test_shrinking_sphere_area_falls_linearly():
    N, sigma, steps = 64, 2.0, 10
    o = Oracle(ball_labels((N, N, N), 16.0), 8.0, G=2)
    dt = config_dt(sigma, N)
    o.step(dt)
    areas, r2 = [], []
    for s in range(steps + 1):
        if s:
            o.step(dt)
        areas.append(o.areas()[0][1])
        r2.append((3.0 * o.volumes()[1] / (4.0 * np.pi)) ** (2.0 / 3.0))
    n = np.arange(steps + 1, dtype=float)
    pa = np.polyfit(n, areas, 1)
    resid = np.array(areas) - np.polyval(pa, n)
    assert 1.0 - resid.var() / np.var(areas) > 0.999
    kappa = -np.polyfit(n, r2, 1)[0] / (2.0 * sigma ** 2)
    assert abs(pa[0] / (-8.0 * np.pi * kappa * sigma ** 2) - 1.0) < 0.05, (pa[0], kappa)


def test_bicrystal_weighted_area_is_read_shockley():
    N, W = 48, 6.0
    o = Oracle(np.zeros((N, N, N), np.int32), W, G=2)
    _slab_state(o, N, 10.25, 30.6, W, 3)
    th, thc = 10.0, 15.0
    h = np.radians(th) / 2.0
    quat = np.array([[1.0, 0.0, 0.0, 0.0], [np.cos(h), 0.0, 0.0, np.sin(h)]])
    o.set_physics(1, quat=quat, theta_c_deg=thc)
    a, w = o.areas()
    r = th / thc
    assert np.allclose(w, r * (1.0 - np.log(r)) * a, rtol=1e-12, atol=0)


def test_boundary_energy_falls_every_step():
    c = make_config(1)
    o = Oracle(c["labels"], c["W"], G=c["G"])
    E = [0.5 * o.areas()[0].sum()]
    for _ in range(c["steps"]):
        o.step(c["dt"])
        E.append(0.5 * o.areas()[0].sum())
    assert np.all(np.diff(E) < 0), E
