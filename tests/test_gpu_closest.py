"""Closest grain-boundary-point correction weights on the GPU
(GG_FLAG_CLOSEST_POINT, sec. 3.2 with the correction of sec. 2.1.4) against
the oracle's brute-force mapping: the weight map of every grain equals the
oracle's (FP64: the same pieces, distances and ties; the pair weights differ
only by the rounding of the device transcendentals), FP64 trajectories stay
within 1e-10 in 2D and 3D (also with boxes that take a whole periodic axis),
batched steps equal plain ones, and FP32 weights from the oracle's state agree
outside near-ties."""
import numpy as np
import pytest

from _compare import compare_states
from oracle import Oracle
from synth import config_dt, power_labels, shoemake_quaternions, uniform_voronoi
from test_gpu_io import _same

pytestmark = pytest.mark.gpu

TOL = 1e-10
TUBE = 2.0


def _inputs(dim, N, G, seed):
    rng = np.random.default_rng(seed)
    n = (N, N) if dim == 2 else (N, N, N)
    labels = power_labels(n, uniform_voronoi(n, G, rng))
    return labels, shoemake_quaternions(G, rng)


def _pair(labels, q, W, G, precision="fp64", **kw):
    import paper_1701_06658_amd as gg
    o = Oracle(labels, W, G=G)
    o.set_physics(1, quat=q, theta_c_deg=15.0)
    o.set_closest_point(True, TUBE)
    s = gg.Simulation(labels, W, G=G, precision=precision, physics=gg.PHYS_MISORIENTATION, quat=q,
                      theta_c_deg=15.0, closest_point=True, **kw)
    return o, s


def _weight_diff(o, s, G):
    """Largest |w_oracle - w_gpu|, the number of voxels that differ by more
    than 1e-12, and the voxel count."""
    gw = s.closest_weights()
    worst, nbad, n = 0.0, 0, 0
    for k in range(G):
        alive, lo, ext = o.box(k)
        assert alive == bool(gw["alive"][k]), k
        if not alive:
            continue
        d = np.abs(o.closest_weights(k) - gw["phi"][k])
        worst = max(worst, float(d.max()))
        nbad += int((d > 1e-12).sum())
        n += d.size
    return worst, nbad, n


def _weights_equal(o, s, G, tag, atol=1e-12):
    worst, nbad, n = _weight_diff(o, s, G)
    print(f"[{tag}] weight maps: max |dw| = {worst:.3e} over {n} voxels", flush=True)
    assert worst <= atol, tag


def _oracle_of_gpu_state(labels, q, W, G, s):
    """An oracle holding the GPU's current state: functions and ID-field."""
    st = s.state()
    b, iv = s.iota()
    o = Oracle(labels, W, G=G)
    o.set_physics(1, quat=q, theta_c_deg=15.0)
    o.set_closest_point(True, TUBE)
    for k in range(G):
        if not st["alive"][k]:
            o.set_grain(k, False)
            continue
        e = b["ext"][k]
        off = int(b["offset"][k])
        io = iv[off:off + int(np.prod(e))].reshape(int(e[2]), int(e[1]), int(e[0]))
        o.set_grain(k, True, st["lo"][k], st["ext"][k], st["phi"][k], io)
    return o


def _check(o, s, W, tag):
    r = compare_states(o.state(), s.state(), o.n, W)
    print(f"[{tag}] max|dphi|={r['max_abs']:.3e} alive_mismatch={r['alive_mismatch']}", flush=True)
    assert r["alive_mismatch"] == 0 and r["max_abs"] <= TOL, (tag, r)


@pytest.mark.parametrize("dim,N,G,W,sigma,steps", [(2, 96, 30, 6.0, 1.5, 6), (3, 48, 60, 6.0, 1.5, 3)])
def test_weights_and_trajectory_fp64(dim, N, G, W, sigma, steps):
    labels, q = _inputs(dim, N, G, 21 + dim)
    o, s = _pair(labels, q, W, G)
    _weights_equal(o, s, G, f"{dim}D create")
    dt = config_dt(sigma, N)
    for i in range(1, steps + 1):
        o.step(dt)
        s.step(dt)
        _check(o, s, W, f"{dim}D closest step {i}")
    # the mapping of the GPU's own state equals the oracle's mapping of it
    _weights_equal(_oracle_of_gpu_state(labels, q, W, G, s), s, G, f"{dim}D after {steps} steps, own state")
    # against the oracle's trajectory, whose functions differ by ~1e-14 (the
    # device's transcendentals in the pair weights): a piece that wins by less
    # than that, or a node that changes sign, may pick another weight
    worst, nbad, n = _weight_diff(o, s, G)
    print(f"[{dim}D after {steps} steps, oracle trajectory] {nbad} of {n} voxels differ "
          f"(max |dw| = {worst:.3e})", flush=True)
    assert nbad <= 1e-4 * n


def test_whole_axis_boxes_fp64():
    # few grains on a small grid: boxes take whole periodic axes, cells wrap
    labels, q = _inputs(3, 36, 6, 5)
    o, s = _pair(labels, q, 6.0, 6)
    ext = np.array([o.box(k)[2] for k in range(6)])
    assert (ext == 36).any()
    _weights_equal(o, s, 6, "whole axes create")
    dt = config_dt(1.5, 36)
    for i in range(1, 4):
        o.step(dt)
        s.step(dt)
        _check(o, s, 6.0, f"whole axes step {i}")
    _weights_equal(_oracle_of_gpu_state(labels, q, 6.0, 6, s), s, 6, "whole axes, own state")


def test_batched_equals_plain():
    labels, q = _inputs(3, 48, 60, 8)
    _, a = _pair(labels, q, 6.0, 60, batched=True)
    _, b = _pair(labels, q, 6.0, 60)
    dt = config_dt(1.5, 48)
    a.step(dt, 4)
    for _ in range(4):
        b.step(dt)
    _same(a.state(), b.state())
    wa, wb = a.closest_weights(), b.closest_weights()
    for k in range(60):
        if wa["alive"][k]:
            assert np.array_equal(wa["phi"][k], wb["phi"][k])


def test_fp32_weights_from_the_oracle_state():
    # the FP32 simulation loaded with the oracle's state: the same pieces up to
    # FP32 rounding of phi, so the closest piece agrees except at near-ties
    labels, q = _inputs(3, 48, 60, 13)
    o, s = _pair(labels, q, 6.0, 60, precision="fp32")
    dt = config_dt(1.5, 48)
    o.step(dt, 2)
    st = o.state()
    iotas = [o.iota(k) if st["alive"][k] else None for k in range(60)]
    s.load_state(st["alive"], st["lo"], st["ext"], st["phi"], iotas)
    gw = s.closest_weights()
    same = total = 0
    for k in range(60):
        if not st["alive"][k]:
            continue
        ow = o.closest_weights(k)
        d = np.abs(ow - gw["phi"][k])
        same += int((d <= 1e-5).sum())
        total += d.size
    print(f"[fp32] weights within 1e-5 of the oracle's on {same / total:.5f} of {total} voxels", flush=True)
    assert same / total >= 0.999


def test_closest_point_needs_the_misorientation_weights():
    import paper_1701_06658_amd as gg
    labels, q = _inputs(2, 64, 10, 3)
    with pytest.raises(gg.GGError, match="GG_E_ARG"):
        gg.Simulation(labels, 6.0, G=10, precision="fp64", closest_point=True)
