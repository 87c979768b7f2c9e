"""Pins of the oracle's closest grain-boundary-point mapping (sec. 3.2 with the
correction of sec. 2.1.4): the zero level set of each grain's function is cut
into linear pieces (cells split along their main diagonal into triangles /
tetrahedra), every voxel of the tube |phi| < tube takes the weight of the
closest piece, and a piece's weight is the mean pair weight over the distinct
ID-field entries at its cell's nodes.

* planes: for a linear function the pieces lie exactly on its zero plane, so
  the squared distance of every voxel whose foot point lies inside the box is
  phi^2 / |grad phi|^2 (axis-aligned and oblique planes, 2D and 3D);
* sphere: distances within the linearisation error of |R - |x - c||;
* brute force on tiny random boxes: the distance to the zero set of the
  piecewise-linear interpolant found by dense sampling of every cell (no
  pieces, no marching tables), 2D and 3D, and across a whole periodic axis;
* weights: a bicrystal gives the pair weight at every tube voxel; a
  tricrystal gives the mean of the two pair weights exactly on the pieces of
  the junction cells; with a tube wider than the band a bicrystal's step
  equals the ID-field step (there both name the one neighbour);
* the ID-field against the closest point on a 2D and a 3D microstructure:
  the share of tube voxels whose weights agree, and the disagreements lie
  next to junctions.
"""
import itertools

import numpy as np
import pytest

from oracle import Oracle, closest_box, pair_weight, misorientation_deg
from synth import config_dt, power_labels, shoemake_quaternions, uniform_voronoi


def _linear_box(ext, grad, c0):
    ex, ey, ez = ext
    z, y, x = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
    return c0 + grad[0] * x + grad[1] * y + grad[2] * z, (x, y, z)


@pytest.mark.parametrize("grad,c0", [((0.0, 0.0, -1.0), 5.3), ((0.31, -0.55, 0.77), -2.2),
                                     ((-0.6, 0.25, 0.4), 1.1)])
def test_plane_3d(grad, c0):
    ext, n = (12, 11, 13), (40, 40, 40)
    f, (x, y, z) = _linear_box(ext, grad, c0)
    d2, cell, piece = closest_box(f, n, 2.0)
    g2 = float(np.dot(grad, grad))
    tube = np.abs(f) < 2.0
    # the foot point x - f grad / |grad|^2 must lie inside the box's cells
    foot = [c - f * g / g2 for c, g in zip((x, y, z), grad)]
    inner = tube & np.all([(p >= 0) & (p <= e - 1) for p, e in zip(foot, ext)], axis=0)
    assert inner.sum() > 200
    assert np.all(d2[tube] >= 0) and np.all(d2[~tube] == -1)
    assert np.allclose(d2[inner], f[inner] ** 2 / g2, rtol=0, atol=1e-12)
    assert np.all(d2[tube] >= f[tube] ** 2 / g2 - 1e-12)      # never nearer than the plane


def test_plane_2d():
    ext, n = (15, 14, 1), (40, 40, 1)
    grad = (0.8, -0.45, 0.0)
    f, (x, y, _) = _linear_box(ext, grad, 0.3 + 3.0)
    d2, _, _ = closest_box(f[0], n[:2], 2.5)
    d2 = d2[0]
    g2 = grad[0] ** 2 + grad[1] ** 2
    tube = np.abs(f[0]) < 2.5
    fx, fy = x[0] - f[0] * grad[0] / g2, y[0] - f[0] * grad[1] / g2
    inner = tube & (fx >= 0) & (fx <= ext[0] - 1) & (fy >= 0) & (fy <= ext[1] - 1)
    assert inner.sum() > 20
    assert np.allclose(d2[inner], f[0][inner] ** 2 / g2, rtol=0, atol=1e-12)


def test_sphere_3d():
    ext, n = (24, 24, 24), (64, 64, 64)
    c, R = np.array([11.3, 12.1, 11.7]), 7.5
    z, y, x = np.meshgrid(np.arange(24), np.arange(24), np.arange(24), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    f = R - r
    d2, _, _ = closest_box(f, n, 2.0)
    tube = np.abs(f) < 2.0
    err = np.abs(np.sqrt(d2[tube]) - np.abs(f[tube]))
    # chords of a sphere of radius R over cells of edge 1 lie within ~3/(8R) of it
    assert err.max() < 3.0 / (8 * R) + 1e-9, err.max()


# ---------------------------------------------------------------- brute force

def _kuhn_value(fc, p):
    """Piecewise-linear interpolant of the corner values fc (indexed by corner
    bits, bit a = axis a) at local points p (m, D) of one cell: the simplex is
    the ordering of the coordinates (Kuhn / Freudenthal), and the value is the
    barycentric combination along the chain of corners it visits."""
    m, D = p.shape
    order = np.argsort(-p, axis=1, kind="stable")          # largest coordinate first
    ps = np.take_along_axis(p, order, 1)
    bits = np.zeros(m, int)
    val = fc[bits] * (1.0 - ps[:, 0])
    for i in range(D):
        bits = bits | (1 << order[:, i])
        w = ps[:, i] - (ps[:, i + 1] if i + 1 < D else 0.0)
        val = val + fc[bits] * w
    return val


def _sampled_zero_set(f, dim, ring, res):
    """Points of the zero set of the piecewise-linear interpolant over every
    cell of the box, by sign changes between neighbouring samples of a res^D
    lattice per cell (linear interpolation between the two samples)."""
    e = f.shape[::-1][:dim]
    cells = [range(e[a] if ring[a] else e[a] - 1) for a in range(dim)]
    g = np.linspace(0.0, 1.0, res)
    lat = np.stack(np.meshgrid(*([g] * dim), indexing="ij"), -1)   # (res,)*D + (D,)
    pts = []
    for c in itertools.product(*cells):
        fc = np.empty(1 << dim)
        for b in range(1 << dim):
            idx = [(c[a] + ((b >> a) & 1)) % e[a] for a in range(dim)]
            fc[b] = f[tuple(idx[::-1])] if dim == 3 else f[idx[1], idx[0]]
        if (fc > 0).all() or (fc <= 0).all():
            continue
        v = _kuhn_value(fc, lat.reshape(-1, dim)).reshape(lat.shape[:-1])
        for a in range(dim):
            sl0 = [slice(None)] * dim
            sl1 = [slice(None)] * dim
            sl0[a] = slice(0, -1)
            sl1[a] = slice(1, None)
            v0, v1 = v[tuple(sl0)], v[tuple(sl1)]
            m = (v0 > 0) != (v1 > 0)
            if not m.any():
                continue
            t = v0[m] / (v0[m] - v1[m])
            p0, p1 = lat[tuple(sl0)][m], lat[tuple(sl1)][m]
            pts.append(np.asarray(c, float) + p0 + t[:, None] * (p1 - p0))
    return np.concatenate(pts)


@pytest.mark.parametrize("dim,ring", [(2, (False, False)), (3, (False, False, False)), (2, (True, False)),
                                      (3, (False, False, True))])
def test_brute_force_tiny_boxes(dim, ring):
    rng = np.random.default_rng(5 + dim + 2 * sum(ring))
    e = [8 if ring[0] else 5, 4, 8 if dim == 3 and ring[2] else 5][:dim]
    # the oracle takes one image of a cell on a whole periodic axis (lower node
    # within half the axis); a piece nearer than e/2 - 1 is seen by it
    far = min([e[a] / 2.0 - 1.0 for a in range(dim) if ring[a]] or [np.inf])
    n = [e[a] if ring[a] else 40 for a in range(dim)]
    shape = tuple(e[::-1])
    f = rng.uniform(-1.5, 1.5, size=shape)
    res = 41 if dim == 2 else 25
    Z = _sampled_zero_set(f, dim, ring, res)
    d2 = closest_box(f, n, 10.0)[0].reshape(shape)
    checked = 0
    for idx in np.ndindex(*shape):
        x = np.array(idx[::-1], float)
        d = Z - x
        for a in range(dim):
            if ring[a]:
                d[:, a] = (d[:, a] + e[a] / 2.0) % e[a] - e[a] / 2.0
        ds = np.sqrt((d ** 2).sum(1)).min()
        do = np.sqrt(d2[idx])
        if do >= far:
            continue   # a piece near the antipode of a whole periodic axis: one image only
        # a sampled point lies within a lattice step of the zero set (on the
        # lattice edge it was found on), and the exact closest point has one
        # within a lattice cell's diagonal
        h = 1.0 / (res - 1)
        assert ds >= do - h - 1e-12, (idx, ds, do)
        assert ds <= do + h * np.sqrt(dim) + 1e-12, (idx, ds, do)
        checked += 1
    assert checked >= 0.8 * np.prod(shape)


# ------------------------------------------------------------------- weights

def _bicrystal(N=20, axis_pos=(6, 14)):
    lab = np.zeros((N, N, N), np.int32)
    lab[:, :, axis_pos[0]:axis_pos[1]] = 1
    return lab


def test_bicrystal_weights_and_step():
    lab = _bicrystal()
    rng = np.random.default_rng(3)
    q = shoemake_quaternions(2, rng)
    w01 = pair_weight(misorientation_deg(q[0], q[1]))[0]
    dt = config_dt(1.0, 20)
    a = Oracle(lab, 3.0, G=2)
    b = Oracle(lab, 3.0, G=2)
    for o in (a, b):
        o.set_physics(1, quat=q, theta_c_deg=15.0)
    b.set_closest_point(True, tube=4.0)              # every voxel of the band
    for k in range(2):
        w = b.closest_weights(k)
        io = b.iota(k)
        assert np.all(w[io >= 0] == w01), k
    a.step(dt, 2)
    b.step(dt, 2)
    for k in range(2):
        assert np.array_equal(a.phi(k), b.phi(k))


def test_tricrystal_junction_weights():
    N = 32
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    ang = np.arctan2(y - 15.7, x - 16.2)
    lab = np.where(ang < -1.0, 0, np.where(ang < 1.3, 1, 2)).astype(np.int32)
    q = shoemake_quaternions(3, np.random.default_rng(9))
    o = Oracle(lab, 6.0, G=3)
    o.set_physics(1, quat=q, theta_c_deg=15.0)
    o.set_closest_point(True, tube=2.0)
    pw = {(i, j): pair_weight(misorientation_deg(q[i], q[j]))[0] for i in range(3) for j in range(3) if i != j}
    for k in range(3):
        alive, lo, ext = o.box(k)
        phi, io, w = o.phi(k), o.iota(k), o.closest_weights(k)
        d2, cell, _ = closest_box(phi, (N, N, N), 2.0)
        tube = np.abs(phi) < 2.0
        others = [j for j in range(3) if j != k]
        mean = (pw[(k, others[0])] + pw[(k, others[1])]) / 2.0
        allowed = {pw[(k, others[0])], pw[(k, others[1])], mean}
        assert set(np.unique(w[tube])) <= allowed
        # the cell of each tube voxel's closest piece decides: one label -> that
        # pair, both labels -> the mean
        ex, ey = ext[0], ext[1]
        n_mean = 0
        for v in zip(*np.nonzero(tube)):
            c = int(cell[v])
            cx, cy, cz = c % ex, (c // ex) % ey, c // (ex * ey)
            labs = {int(io[(cz + dz) % ext[2], (cy + dy) % ext[1], (cx + dx) % ext[0]])
                    for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)}
            labs.discard(-1)
            want = np.mean([pw[(k, j)] for j in sorted(labs)]) if labs else 1.0
            assert w[v] == pytest.approx(want, rel=1e-15, abs=0), (k, v, labs)
            n_mean += len(labs) == 2
        assert n_mean > 10, n_mean                     # the triple line is seen
        # away from the tube: the ID-field pair
        outside = (~tube) & (io >= 0)
        assert np.all(w[outside] == np.vectorize(lambda j: pw[(k, j)])(io[outside]))


@pytest.mark.parametrize("dim", [2, 3])
def test_id_field_against_closest_point(dim):
    """The ID-field names the grain across the closest boundary point for most
    tube voxels; where the closest piece's cell holds more than one neighbour
    (a junction) the two weights part."""
    N, G = (96, 30) if dim == 2 else (40, 40)
    rng = np.random.default_rng(11)
    n = (N, N) if dim == 2 else (N, N, N)
    labels = power_labels(n, uniform_voronoi(n, G, rng))
    q = shoemake_quaternions(G, rng)
    o = Oracle(labels, 6.0, G=G)
    o.set_physics(1, quat=q, theta_c_deg=15.0)
    o.set_closest_point(True, tube=2.0)
    o.step(config_dt(1.5, N), 2)
    agree = total = 0
    for k in range(G):
        alive, lo, ext = o.box(k)
        if not alive:
            continue
        phi, io, w = o.phi(k), o.iota(k), o.closest_weights(k)
        tube = (np.abs(phi) < 2.0) & (io >= 0)
        wid = np.vectorize(lambda j: pair_weight(misorientation_deg(q[k], q[j]))[0])(io[tube])
        total += int(tube.sum())
        agree += int((w[tube] == wid).sum())
    share = agree / total
    print(f"[{dim}D] closest-point and ID-field weights agree on {share:.4f} of {total} tube voxels")
    assert total > 5000 and share > 0.85
