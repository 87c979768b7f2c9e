"""Label fields for periodic grids: Voronoi / power diagrams and simple shapes.

Conventions shared by every consumer:
  * a label field is an ``int32`` array of shape ``(nz, ny, nx)`` (``nz == 1``
    in 2D), so that the flat index is ``x + nx*(y + ny*z)`` (x fastest);
  * voxel ``i`` along an axis has its centre at ``i + 0.5``;
  * grain ids are ``0 .. G-1``.

Power-diagram labels are exact in FP64: voxel ``x`` belongs to
``argmin_k (sum_a d_a^2 - w_k)`` with the periodic minimum-image difference
``d_a = x_a - s_{k,a} - N_a*round((x_a - s_{k,a})/N_a)``, the squares summed in
axis order x, y, z, and ties going to the lowest ``k``.  A k-d tree proposes
the few nearest candidates; the exact score above then decides among them.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def _grid_shape(n):
    n = tuple(int(v) for v in n)
    if len(n) == 2:
        n = (n[0], n[1], 1)
    if len(n) != 3 or min(n) < 1:
        raise ValueError(f"bad grid {n}")
    return n  # (nx, ny, nz)


def power_labels(n, seeds, weights=None, k_check=4, slab_voxels=1 << 22):
    """Exact periodic power-diagram labels (plain Voronoi when ``weights`` is None)."""
    nx, ny, nz = _grid_shape(n)
    dim = 2 if nz == 1 else 3
    seeds = np.asarray(seeds, dtype=np.float64)
    G = seeds.shape[0]
    if seeds.shape != (G, dim):
        raise ValueError("seeds must be (G, dim)")
    w = np.zeros(G) if weights is None else np.asarray(weights, dtype=np.float64)
    box = np.array([nx, ny, nz][:dim], dtype=np.float64)
    s = np.mod(seeds, box)
    s[s >= box] = 0.0
    wmax = float(w.max()) if G else 0.0
    lift = np.sqrt(np.maximum(wmax - w, 0.0))
    data = np.concatenate([s, lift[:, None]], axis=1)
    lbox = np.concatenate([box, [2.0 * float(lift.max() if G else 0.0) + 1.0]])
    tree = cKDTree(data, boxsize=lbox)
    k = min(k_check, G)
    out = np.empty((nz, ny, nx), dtype=np.int32)
    plane = nx * ny
    zstep = max(1, slab_voxels // plane)
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    for z0 in range(0, nz, zstep):
        z1 = min(nz, z0 + zstep)
        cnt = (z1 - z0) * plane
        q = np.empty((cnt, dim + 1))
        q[:, 0] = np.tile(xx.ravel(), z1 - z0)
        q[:, 1] = np.tile(yy.ravel(), z1 - z0)
        if dim == 3:
            q[:, 2] = np.repeat(np.arange(z0, z1) + 0.5, plane)
        q[:, dim] = 0.0
        _, cand = tree.query(q, k=k, workers=-1)
        cand = cand.reshape(cnt, k)
        score = None
        for a in range(dim):
            diff = q[:, a:a + 1] - s[cand, a]
            diff = diff - box[a] * np.round(diff / box[a])
            sq = diff * diff
            score = sq if score is None else score + sq
        score = score - w[cand]
        # ties -> lowest id
        best = np.empty(cnt, dtype=np.int64)
        bsc = score[:, 0].copy()
        best[:] = cand[:, 0]
        for c in range(1, k):
            sc = score[:, c]
            cd = cand[:, c]
            take = (sc < bsc) | ((sc == bsc) & (cd < best))
            bsc = np.where(take, sc, bsc)
            best = np.where(take, cd, best)
        out[z0:z1] = best.reshape(z1 - z0, ny, nx).astype(np.int32)
    return out


def compact_labels(labels):
    """Renumber the non-empty labels to ``0..G'-1`` keeping their order."""
    ids, inv = np.unique(labels, return_inverse=True)
    return inv.reshape(labels.shape).astype(np.int32), ids


def uniform_voronoi(n, G, rng):
    """Seeds uniform on the periodic box (plain Voronoi, zero weights)."""
    nx, ny, nz = _grid_shape(n)
    dim = 2 if nz == 1 else 3
    box = np.array([nx, ny, nz][:dim], dtype=np.float64)
    return rng.random((G, dim)) * box


def rsa_power_diagram(n, radii, rng, packing=0.3, max_tries=2000):
    """Random sequential addition of non-overlapping periodic balls.

    Ball radii are ``c*radii`` with ``c`` chosen so that the balls fill the
    given volume fraction; they are placed largest first at uniform random
    positions, rejecting overlaps.  Returns ``(seeds, weights)`` with power
    weights ``w_k = (c*r_k)^2``: every power cell then contains its ball.
    """
    nx, ny, nz = _grid_shape(n)
    dim = 2 if nz == 1 else 3
    box = np.array([nx, ny, nz][:dim], dtype=np.float64)
    r = np.asarray(radii, dtype=np.float64)
    vol = float(np.prod(box))
    unit = np.pi * (r ** 2).sum() if dim == 2 else (4.0 / 3.0) * np.pi * (r ** 3).sum()
    c = (packing * vol / unit) ** (1.0 / dim)
    rad = c * r
    order = np.argsort(-rad, kind="stable")
    cell = 2.0 * float(rad.max())
    ncell = np.maximum(1, np.floor(box / cell).astype(int))
    csize = box / ncell
    grid = {}
    pos = np.zeros((len(r), dim))
    for idx in order:
        ri = rad[idx]
        for _ in range(max_tries):
            p = rng.random(dim) * box
            ci = np.floor(p / csize).astype(int) % ncell
            near = []
            rng_cells = [range(-1, 2)] * dim
            for off in np.array(np.meshgrid(*rng_cells, indexing="ij")).reshape(dim, -1).T:
                key = tuple(((ci + off) % ncell).tolist())
                near.extend(grid.get(key, ()))
            if near:
                near = np.unique(np.array(near))
                d = p[None, :] - pos[near]
                d -= box * np.round(d / box)
                dist2 = (d * d).sum(axis=1)
                if np.any(dist2 < (ri + rad[near]) ** 2):
                    continue
            pos[idx] = p
            grid.setdefault(tuple(ci.tolist()), []).append(idx)
            break
        else:
            raise RuntimeError("random sequential addition did not converge")
    return pos, rad ** 2


def ball_labels(n, radius, centre=None):
    """Grain 1 = voxels whose centre lies strictly inside the ball; grain 0 = the rest."""
    nx, ny, nz = _grid_shape(n)
    dim = 2 if nz == 1 else 3
    if centre is None:
        centre = [nx / 2.0, ny / 2.0, nz / 2.0][:dim]
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5,
                          np.arange(nx) + 0.5, indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2
    if dim == 3:
        r2 = r2 + (z - centre[2]) ** 2
    return (r2 < radius * radius).astype(np.int32)


def slab_labels(n, normal, offset, width):
    """Grain 1 = the periodic slab ``0 <= (normal.x - offset) mod P < width``.

    ``normal`` must have integer components so that the slab is compatible with
    the periodic box; ``P`` is the period of ``normal.x`` (the grid size when the
    sizes are equal).  Grain 0 = the rest.
    """
    nx, ny, nz = _grid_shape(n)
    dim = 2 if nz == 1 else 3
    nv = np.asarray(normal, dtype=np.int64)
    if nv.shape != (dim,):
        raise ValueError("normal must have dim integer components")
    period = int(np.gcd.reduce([int(abs(v)) * s for v, s in zip(nv, (nx, ny, nz)) if v != 0]))
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5,
                          np.arange(nx) + 0.5, indexing="ij")
    proj = nv[0] * x + nv[1] * y + (nv[2] * z if dim == 3 else 0.0)
    t = np.mod(proj - offset, period)
    return (t < width).astype(np.int32)


def shoemake_quaternions(G, rng):
    """Uniform random rotations (Shoemake's method), ``(G, 4)`` as (w, x, y, z)."""
    u = rng.random((G, 3))
    a = np.sqrt(1.0 - u[:, 0])
    b = np.sqrt(u[:, 0])
    t1 = 2.0 * np.pi * u[:, 1]
    t2 = 2.0 * np.pi * u[:, 2]
    return np.stack([b * np.cos(t2), a * np.sin(t1), a * np.cos(t1), b * np.sin(t2)], axis=1)


def random_unit_vectors(G, rng, dim=3):
    """Directions uniform on the unit sphere, ``(G, dim)``."""
    v = rng.standard_normal((G, dim))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


MU0 = 4.0e-7 * np.pi  # vacuum permeability, T m / A


def magnetic_energy_density(c_axis, field_dir, delta_chi, B_tesla):
    """Orientation-dependent magnetic energy density of each grain, J/m^3.

    ``E = delta_chi * B^2 * cos^2(theta) / (2 mu0)`` with ``theta`` the angle
    between the grain's c-axis and the field; the orientation-independent
    ``chi_perp`` part is dropped since only differences drive the boundaries.
    """
    c = np.asarray(c_axis, dtype=np.float64)
    f = np.asarray(field_dir, dtype=np.float64)
    f = f / np.linalg.norm(f)
    cos = (c @ f) / np.linalg.norm(c, axis=1)
    return delta_chi * B_tesla ** 2 * cos ** 2 / (2.0 * MU0)
