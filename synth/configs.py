"""The five synthetic workloads of the grain-growth step, seeded and cached.

Each workload stands in for the paper's private microstructures: Voronoi
starts of a few thousand to fifty thousand grains on a periodic cube (or a 2D
square), with the Gaussian width ``sigma`` and the narrow-band width ``W`` in
voxels.  The normalised time step that gives ``sigma`` on an ``N``-voxel grid is
``dt = sigma^2 / (2 N^2)`` (the heat kernel has variance ``2 dt`` per axis in
units where the domain is the unit cube).

Random streams: ``numpy.random.default_rng(1701066580 + index)`` (PCG64); the
seed points are drawn first, then any orientation data.
"""
from __future__ import annotations

import os

import numpy as np

from .labels import (compact_labels, magnetic_energy_density, power_labels,
                     random_unit_vectors, rsa_power_diagram, shoemake_quaternions,
                     uniform_voronoi)

SEED_BASE = 1701066580

CONFIGS = {
    1: dict(name="2d-64sq-20grains-fp64", dim=2, N=64, G=20, sizes="uniform",
            sigma=1.5, W=6.0, steps=20, precision="fp64"),
    2: dict(name="3d-128cube-1000grains-fp64", dim=3, N=128, G=1000, sizes="uniform",
            sigma=2.0, W=8.0, steps=50, precision="fp64"),
    3: dict(name="3d-256cube-8000grains-lognormal-mixed", dim=3, N=256, G=8000,
            sizes="lognormal", sigma=2.0, W=8.0, steps=100, precision="fp32"),
    4: dict(name="3d-512cube-50000grains-aniso-fp32", dim=3, N=512, G=50000,
            sizes="uniform", sigma=2.0, W=8.0, steps=100, precision="fp32",
            physics="anisotropic"),
    5: dict(name="3d-512cube-50000grains-bimodal-magnetic", dim=3, N=512, G=50000,
            sizes="bimodal", sigma=2.0, W=8.0, steps=200, precision="fp32",
            physics="magnetic"),
}


def config_dt(sigma, N):
    """Normalised time step whose heat kernel has standard deviation ``sigma`` voxels."""
    return float(sigma) ** 2 / (2.0 * float(N) ** 2)


def _cache_dir():
    d = os.environ.get("GG_SYNTH_CACHE") or os.path.join(
        os.environ.get("TMPDIR", "/tmp"), "gg_synth_cache")
    os.makedirs(d, exist_ok=True)
    return d


def make_config(index, N=None, G=None, cache=True):
    """Build workload ``index`` (1..5); ``N``/``G`` override the size for scaled cuts.

    Returns a dict with ``labels`` (int32, (nz, ny, nx)), ``G`` (after dropping
    empty power cells and renumbering), ``dim``, ``n`` (nx, ny, nz), ``sigma``,
    ``W``, ``steps``, ``dt``, ``precision`` and, when the workload has physics
    data, ``quat`` ((G, 4) w,x,y,z) or ``c_axis`` ((G, 3)).
    """
    base = dict(CONFIGS[index])
    N = int(N or base["N"])
    G0 = int(G or base["G"])
    dim = base["dim"]
    n = (N, N, N) if dim == 3 else (N, N, 1)
    rng = np.random.default_rng(SEED_BASE + index)
    key = f"cfg{index}_N{N}_G{G0}.npz"
    path = os.path.join(_cache_dir(), key)
    weights = None
    if base["sizes"] == "uniform":
        seeds = uniform_voronoi(n, G0, rng)
    elif base["sizes"] == "lognormal":
        radii = np.exp(rng.normal(0.0, 0.5, size=G0))
        seeds, weights = rsa_power_diagram(n, radii, rng, packing=0.3)
    elif base["sizes"] == "bimodal":
        big = G0 // 20
        radii = np.ones(G0)
        radii[rng.permutation(G0)[:big]] = 4.0
        seeds, weights = rsa_power_diagram(n, radii, rng, packing=0.3)
    else:
        raise ValueError(base["sizes"])
    extra = {}
    if base.get("physics") == "anisotropic":
        extra["quat"] = shoemake_quaternions(G0, rng)
    elif base.get("physics") == "magnetic":
        extra["c_axis"] = random_unit_vectors(G0, rng, 3)
    if cache and os.path.exists(path):
        with np.load(path, allow_pickle=False) as f:
            labels = f["labels"]
            kept = f["kept"]
    else:
        labels = power_labels(n, seeds, weights)
        labels, kept = compact_labels(labels)
        if cache:
            tmp = path + f".tmp{os.getpid()}.npz"
            np.savez(tmp, labels=labels, kept=kept)
            os.replace(tmp, path)
    for k in list(extra):
        extra[k] = np.ascontiguousarray(extra[k][kept])
    out = dict(base)
    out.update(dict(index=index, N=N, n=n, G=int(len(kept)), labels=labels,
                    dt=config_dt(base["sigma"], N), kept=kept, **extra))
    if base.get("physics") == "anisotropic":
        out["theta_c_deg"] = 15.0
    if base.get("physics") == "magnetic":
        # titanium in a 17 T field along z; gamma, mobility and the voxel size
        # chosen so that the mean grain's equivalent-sphere diameter is 20 um
        out["delta_chi"], out["B_tesla"] = 1.18e-5, 17.0
        out["field_dir"] = np.array([0.0, 0.0, 1.0])
        out["energy"] = magnetic_energy_density(out["c_axis"], out["field_dir"],
                                                out["delta_chi"], out["B_tesla"])
        out["gamma_max"], out["mobility_max"] = 0.3, 3.0e-11
        mean_vol = float(np.prod(n)) / out["G"]
        out["h_phys"] = 20.0e-6 / (6.0 * mean_vol / np.pi) ** (1.0 / 3.0)
    return out
