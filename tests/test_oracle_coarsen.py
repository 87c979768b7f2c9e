"""Pins of the oracle's grid coarsening (sec. 3, sequential optimizations: each
function projected onto a coarser grid by trilinear interpolation, the grid
spacing growing as grains vanish):

* the remap of a box function against SciPy's periodic linear interpolation of
  the same function on the whole grid (-W outside the box), divided by r;
* an oblique periodic slab array whose functions are exact taxicab distances:
  linear interpolation keeps the interface exactly, so the coarsened functions
  are the exact taxicab distances on the new grid (r = 2 and r = 4/3);
* an integer ratio keeps every grain's positive set on the new nodes, so the
  labels are the old labels at the nodes i' r; volumes sum to the new grid;
* a grain smaller than the new spacing vanishes;
* the bulk term after coarsening moves a flat boundary by the displacement of
  the new voxel edge r h.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import Oracle, coarse_sample_box
from synth import config_dt, make_config
from test_oracle_step import _slab_positions, _slab_state


@pytest.mark.parametrize("dim,n,npr", [(3, (20, 20, 20), (15, 15, 15)), (3, (24, 24, 24), (12, 12, 12)),
                                       (2, (30, 30, 1), (18, 18, 1))])
def test_remap_matches_periodic_linear_interpolation(dim, n, npr):
    rng = np.random.default_rng(5)
    W = 3.0
    shape = (n[2], n[1], n[0])
    # a partial box wrapping around x, and a whole-axis box along the others
    lo = np.array([n[0] - 4, 0, 0], np.int32)
    ext = np.array([n[0] // 2, n[1], n[2]], np.int32)
    f = rng.uniform(-W, W, size=(ext[2], ext[1], ext[0]))
    full = np.full(shape, -W)
    zs = (np.arange(ext[2]) + lo[2]) % n[2]
    ys = (np.arange(ext[1]) + lo[1]) % n[1]
    xs = (np.arange(ext[0]) + lo[0]) % n[0]
    full[np.ix_(zs, ys, xs)] = f
    r = n[0] / npr[0]
    new_lo = np.array([3, 1, 0], np.int32)
    new_ext = np.array([npr[0] - 2, npr[1] - 3, npr[2]], np.int32)
    out = coarse_sample_box(f, W, n, npr, lo, new_lo, new_ext, dim=dim)
    gz = (np.arange(new_ext[2]) + new_lo[2]) % npr[2]
    gy = (np.arange(new_ext[1]) + new_lo[1]) % npr[1]
    gx = (np.arange(new_ext[0]) + new_lo[0]) % npr[0]
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    if dim == 3:
        coords = np.stack([Z * r, Y * r, X * r])
        ref = ndimage.map_coordinates(full, coords.reshape(3, -1), order=1, mode="grid-wrap")
    else:
        coords = np.stack([Y * r, X * r])
        ref = ndimage.map_coordinates(full[0], coords.reshape(2, -1), order=1, mode="grid-wrap")
    ref = ref.reshape(out.shape) / r
    assert np.max(np.abs(out - ref)) < 1e-12


def _slab_field(N, d, L, c, dim, r=1.0):
    """Exact taxicab distance (in voxels of a grid with spacing r) to the planes
    d.x = c + k L (unit ||d||_inf), positive inside alternate slabs."""
    ax = np.arange(N, dtype=float) * r
    if dim == 3:
        z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
        s = d[0] * x + d[1] * y + d[2] * z - c
    else:
        y, x = np.meshgrid(ax, ax, indexing="ij")
        s = (d[0] * x + d[1] * y - c)[None]
    return (L / 4.0 - np.abs(np.mod(s, L) - L / 2.0)) / r


@pytest.mark.parametrize("dim,Np", [(3, 24), (3, 36), (2, 24), (2, 36)])
def test_coarsened_slab_array_is_exact(dim, Np):
    N, W, L = 48, 4.0, 24.0
    d = np.array([0.5, 1.0, 1.0]) if dim == 3 else np.array([0.5, 1.0])
    f = _slab_field(N, d, L, 0.37, dim)
    shape = (N, N, N) if dim == 3 else (1, N, N)
    labels = (f <= 0).astype(np.int32).reshape(shape)
    o = Oracle(labels, W, G=2)
    ext = [N, N, N if dim == 3 else 1]
    o.set_grain(0, True, [0, 0, 0], ext, np.clip(f, -W, W))
    o.set_grain(1, True, [0, 0, 0], ext, np.clip(-f, -W, W))
    o.coarsen((Np, Np, Np if dim == 3 else 1))
    r = N / Np
    g = _slab_field(Np, d, L, 0.37, dim, r)
    for k, sgn in ((0, 1.0), (1, -1.0)):
        alive, lo, e = o.box(k)
        assert alive and list(e[:dim]) == [Np] * dim
        assert np.max(np.abs(o.phi(k) - np.clip(sgn * g, -W, W))) < 1e-12
    assert abs(o.volumes().sum() - Np ** dim) < 1e-9 * Np ** dim


@pytest.mark.parametrize("dim", [2, 3])
def test_integer_ratio_keeps_positive_sets(dim):
    c = make_config(1) if dim == 2 else make_config(2, N=72, G=80)
    o = Oracle(c["labels"], c["W"], G=c["G"])
    o.step(c["dt"], 2)
    before = o.labels()
    N = c["N"]
    Np = N // 2
    new = (Np, Np, Np if dim == 3 else 1)
    alive_before = o.alive_count()
    o.coarsen(new)
    after = o.labels()
    sub = before[::2, ::2, ::2] if dim == 3 else before[:, ::2, ::2]
    # a voxel is owned by the grain positive there: positive sets are kept exactly
    st = o.state()
    pos_any = np.zeros(after.shape, bool)
    for k in range(c["G"]):
        if not st["alive"][k]:
            continue
        lo, ext = st["lo"][k], st["ext"][k]
        zs = (np.arange(ext[2]) + lo[2]) % after.shape[0]
        ys = (np.arange(ext[1]) + lo[1]) % after.shape[1]
        xs = (np.arange(ext[0]) + lo[0]) % after.shape[2]
        pos_any[np.ix_(zs, ys, xs)] |= st["phi"][k] > 0
    assert np.array_equal(after[pos_any], sub[pos_any])
    assert pos_any.mean() > 0.8
    assert o.alive_count() <= alive_before
    V = o.volumes()
    assert abs(V.sum() - Np ** dim) < 5e-3 * Np ** dim
    # the coarser state keeps stepping with the time step of the new grid
    o.step(config_dt(c["sigma"], Np), 2)
    V = o.volumes()
    assert abs(V.sum() - Np ** dim) < 5e-3 * Np ** dim


def test_small_grain_vanishes():
    N, W = 64, 4.0
    y, x = np.mgrid[0:N, 0:N]
    labels = ((x - 30.5) ** 2 + (y - 30.5) ** 2 < 1.3 ** 2).astype(np.int32)[None]
    o = Oracle(labels, W, G=2)
    assert o.box(1)[0]
    o.coarsen((20, 20, 1))
    assert not o.box(1)[0] and o.box(0)[0]
    assert o.volumes()[1] == 0.0
    assert abs(o.volumes()[0] - 400.0) < 1e-9


def test_bulk_term_uses_the_coarser_voxel_edge():
    # the flat-boundary displacement b = dE sigma^2 h / (2 gamma) per step with
    # h the new voxel edge r h
    N, Np, W, sigma = 128, 64, 6.0, 1.5
    labels = np.zeros((1, N, N), np.int32)
    o = Oracle(labels, W, G=2)
    _slab_state(o, N, 40.0, 81.0, W, 2)   # planes at old x = 40, 81 -> new 20, 40.5
    gam, h = 0.3, 1e-6
    E = np.array([600.0, 150.0])
    o.set_physics(2, energy=E, h_phys=h, gamma_max=gam)
    o.coarsen((Np, Np, 1))
    p0 = _slab_positions(o)
    assert np.allclose(p0, [20.0, 40.5], atol=1e-9)
    b = (E[0] - E[1]) * sigma ** 2 * (h * N / Np) / (2.0 * gam)
    steps = 10
    o.step(config_dt(sigma, Np), steps)
    p = _slab_positions(o)
    moved = np.array([p0[0] - p[0], p[1] - p0[1]]) / steps
    assert np.all(np.abs(moved - b) < 1e-3 * b), (moved, b)
