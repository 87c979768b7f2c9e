"""The seeded input generators (no method arithmetic): exact periodic power
diagrams against brute force, reproducibility, and the size statistics of the
lognormal and bimodal workloads at reduced size."""
import numpy as np
import pytest

from synth import make_config, power_labels, rsa_power_diagram, shoemake_quaternions, uniform_voronoi


def _brute(n, seeds, w):
    nx, ny, nz = n
    dim = seeds.shape[1]
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    pts = [x, y, z][:dim]
    best = np.full(x.shape, np.inf)
    lab = np.zeros(x.shape, np.int32)
    for k in range(len(seeds)):
        s = 0.0
        for a in range(dim):
            d = pts[a] - seeds[k, a]
            d = d - n[a] * np.round(d / n[a])
            s = s + d * d
        s = s - w[k]
        better = s < best                    # strict: ties stay with the lower id
        best[better] = s[better]
        lab[better] = k
    return lab


@pytest.mark.parametrize("n,G,weighted", [((23, 17, 1), 9, False), ((23, 17, 1), 9, True),
                                          ((12, 10, 9), 14, True)])
def test_power_labels_are_the_exact_periodic_power_diagram(n, G, weighted):
    rng = np.random.default_rng(31)
    dim = 2 if n[2] == 1 else 3
    seeds = rng.random((G, dim)) * np.array(n[:dim])
    w = rng.uniform(0, 20, G) if weighted else np.zeros(G)
    got = power_labels(n, seeds, w if weighted else None)
    assert np.array_equal(got, _brute(n, seeds, w))


def test_ties_go_to_the_lowest_id():
    # two coincident seeds with equal weights: the lower id takes every voxel of the pair
    n = (16, 16, 1)
    seeds = np.array([[4.0, 4.0], [12.0, 12.0], [4.0, 4.0]])
    lab = power_labels(n, seeds)
    assert not (lab == 2).any() and (lab == 0).sum() > 50


def test_configs_are_reproducible_and_compact():
    a = make_config(1, cache=False)
    b = make_config(1, cache=False)
    assert np.array_equal(a["labels"], b["labels"]) and a["G"] == b["G"]
    lab = a["labels"]
    assert lab.dtype == np.int32 and lab.shape == (1, 64, 64)
    assert set(np.unique(lab)) == set(range(a["G"]))


def test_lognormal_and_bimodal_size_statistics():
    rng = np.random.default_rng(5)
    n = (64, 64, 64)
    G = 300
    radii = np.exp(rng.normal(0.0, 0.5, G))
    seeds, w = rsa_power_diagram(n, radii, rng, packing=0.3)
    lab = power_labels(n, seeds, w)
    vol = np.bincount(lab.ravel(), minlength=G).astype(float)
    assert np.all(vol > 0)
    r_eq = np.cbrt(vol)
    # the cells follow their drawn radii (lognormal, sigma_ln 0.5), but the
    # space between the balls (70% at packing 0.3) narrows the spread of the
    # cells' equivalent radii to about sigma_ln 0.2
    assert np.corrcoef(np.log(r_eq), np.log(radii))[0, 1] > 0.8
    assert 0.12 < np.std(np.log(r_eq)) < 0.35
    radii = np.ones(G)
    radii[: G // 20] = 4.0
    seeds, w = rsa_power_diagram(n, radii, rng, packing=0.3)
    vol = np.bincount(power_labels(n, seeds, w).ravel(), minlength=G).astype(float)
    assert vol[: G // 20].mean() > 8.0 * np.median(vol[G // 20:])


def test_orientation_and_seed_generators():
    rng = np.random.default_rng(2)
    q = shoemake_quaternions(20000, rng)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0)
    # uniform on SO(3): E[w^2] = 1/4 for each component
    assert np.allclose((q * q).mean(0), 0.25, atol=0.01)
    s = uniform_voronoi((10, 20, 1), 1000, rng)
    assert s.shape == (1000, 2) and s.min() >= 0 and (s.max(0) < [10, 20]).all()
