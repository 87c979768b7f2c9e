"""The device-driven step (through the C ABI): batched steps (captured HIP
graphs, gg_step returning before the steps finish) give the same states as
plain launches and as the oracle; a step whose new boxes or coverage lists do
not fit the device buffers is taken again after the buffers grow (forced from
the host with buffers that hold exactly the current layout); the launch order
of the grains changes no value; a change of dt keeps the separable predictor
consistent; a checkpoint of a finer grid loads into a simulation created on a
coarser one."""
import numpy as np
import pytest

from _compare import compare_states
from oracle import Oracle
from synth import config_dt, make_config
from test_gpu_io import _same

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def _sim(c, precision="fp64", **kw):
    import paper_1701_06658_amd as gg
    return gg.Simulation(c["labels"], c["W"], G=c["G"], precision=precision, **kw)


def _check(o, s, W, tag):
    r = compare_states(o.state(), s.state(), o.n, W)
    print(f"[{tag}] max|dphi|={r['max_abs']:.3e} alive_mismatch={r['alive_mismatch']}", flush=True)
    assert r["alive_mismatch"] == 0 and r["max_abs"] <= TOL_FP64, (tag, r)
    assert np.allclose(o.volumes(), s.volumes(), rtol=1e-10, atol=1e-9), tag


@pytest.mark.parametrize("index,N,G", [(1, None, None), (2, 64, 125)])
def test_batched_equals_plain_and_oracle(index, N, G):
    c = make_config(index, N=N, G=G)
    o = Oracle(c["labels"], c["W"], G=c["G"])
    a = _sim(c, batched=True)
    b = _sim(c, batched=False)
    for chunk in (1, 4, 7):
        a.step(c["dt"], chunk)       # queued: returns before the steps finish
        for _ in range(chunk):
            b.step(c["dt"])
        o.step(c["dt"], chunk)
        _same(a.state(), b.state())
        assert np.array_equal(a.volumes(), b.volumes())
        _check(o, a, c["W"], f"cfg{index} batched after +{chunk}")
    assert a.stats()["steps"] == b.stats()["steps"] == 12
    assert a.stats()["total_grain_voxels"] == b.stats()["total_grain_voxels"]
    assert np.array_equal(a.labels(), o.labels())


@pytest.mark.parametrize("batched", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_exact_buffers_retake_growing_steps(batched, precision):
    # headroom 1: the buffers hold exactly the current layout, so every step
    # whose boxes or coverage lists grow fails its capacity check, leaves its
    # starting state untouched and is taken again after the buffers grow
    c = make_config(2, N=64, G=125)
    a = _sim(c, precision, batched=batched, headroom=1.0)
    b = _sim(c, precision)
    cap0 = a.stats()["capacity"]
    a.step(c["dt"], 10)
    b.step(c["dt"], 10)
    _same(a.state(), b.state())
    assert np.array_equal(a.volumes(), b.volumes())
    assert a.stats()["steps"] == 10
    assert a.stats()["total_grain_voxels"] == b.stats()["total_grain_voxels"]
    print(f"[exact {precision} batched={batched}] capacity {cap0} -> {a.stats()['capacity']}", flush=True)
    if precision == "fp64":
        o = Oracle(c["labels"], c["W"], G=c["G"])
        o.step(c["dt"], 10)
        _check(o, a, c["W"], "exact buffers")


def test_growing_grain_forces_retakes():
    # a grain that grows every step (bulk driving force, fp64) under exact
    # buffers: the retake path runs on most steps, results stay exact
    from test_gpu_parity import _physics_inputs
    import paper_1701_06658_amd as gg
    labels, gphys, ophys = _physics_inputs("bulk")
    G = int(labels.max()) + 1
    W, sigma = 8.0, 2.0
    dt = config_dt(sigma, labels.shape[0])
    o = Oracle(labels, W, G=G)
    o.set_physics(**ophys)
    s = gg.Simulation(labels, W, G=G, precision="fp64", headroom=1.0, batched=True, **gphys)
    s.step(dt, 6)
    o.step(dt, 6)
    _check(o, s, W, "bulk growth, exact buffers")


def growing_disk(dim=2, N=64, r0=10.45, push=1.0, sigma=1.5):
    """A disk (ball) grain 1 in a matrix grain 0 whose bulk energy density is
    higher: the bulk term moves the boundary outward by about `push` voxels a
    step, so grain 1's box grows within a few steps while the matrix keeps its
    whole-axis box: the layout's total volume grows.  Returns labels, the GPU
    and oracle physics arguments and dt."""
    n = (N,) * dim
    c = (N - 1) / 2.0
    g = np.meshgrid(*[np.arange(N)] * dim, indexing="ij")
    r2 = sum((x - c) ** 2 for x in g)
    labels = (r2 < r0 ** 2).astype(np.int32)
    if dim == 2:
        labels = labels[None]
    h, gam = 2.0e-5, 0.3
    scale = sigma ** 2 * h / (2 * gam)            # voxels per (J/m^3) and step
    energy = np.array([push / scale, 0.0])
    gpu = dict(physics=2, energy=energy, voxel_m=h, gamma_max=gam)
    orc = dict(mode=2, energy=energy, h_phys=h, gamma_max=gam)
    return labels, gpu, orc, config_dt(sigma, N)


@pytest.mark.parametrize("dim,batched", [(2, False), (2, True), (3, True)])
def test_growing_disk_forces_retakes(dim, batched):
    # exact buffers: the steps whose layout outgrows them fail their capacity
    # check and are taken again after the buffers grow; the results equal the
    # plain run with headroom and the oracle
    import paper_1701_06658_amd as gg
    labels, gphys, ophys, dt = growing_disk(dim, N=64 if dim == 2 else 40, r0=10.45 if dim == 2 else 7.45)
    W = 6.0
    a = gg.Simulation(labels, W, G=2, precision="fp64", headroom=1.0, batched=batched, **gphys)
    b = gg.Simulation(labels, W, G=2, precision="fp64", **gphys)
    o = Oracle(labels, W, G=2)
    o.set_physics(**ophys)
    cap0 = a.stats()["capacity"]
    a.step(dt, 6)
    b.step(dt, 6)
    o.step(dt, 6)
    cap1 = a.stats()["capacity"]
    print(f"[growing disk {dim}D batched={batched}] capacity {cap0} -> {cap1}", flush=True)
    assert cap1 > cap0                               # the retake path ran
    assert a.stats()["steps"] == 6
    _same(a.state(), b.state())
    _check(o, a, W, f"growing disk {dim}D")


def test_order_size_changes_no_value():
    c = make_config(2, N=64, G=125)
    a = _sim(c, "fp32", batched=True, order_size=True)
    b = _sim(c, "fp32", batched=True, order_size=False)
    a.step(c["dt"], 6)
    b.step(c["dt"], 6)
    _same(a.state(), b.state())
    assert np.array_equal(a.volumes(), b.volumes())


def test_euclid_batched_equals_plain():
    # the Euclidean variant sizes its work items on the host: batched falls back
    # to plain launches, with the same results
    c = make_config(2, N=64, G=125)
    a = _sim(c, "fp64", batched=True, redistance="euclid")
    b = _sim(c, "fp64", redistance="euclid")
    a.step(c["dt"], 3)
    b.step(c["dt"], 3)
    _same(a.state(), b.state())


def test_dt_change_keeps_the_separable_predictor():
    # sigma 2.0 then 1.9 voxels: the same kernel radius R = 8, new taps
    c = make_config(2, N=64, G=125)
    N = c["N"]
    o = Oracle(c["labels"], c["W"], G=c["G"])
    s = _sim(c)
    for sigma in (2.0, 1.9, 1.9, 2.0):
        dt = config_dt(sigma, N)
        o.step(dt)
        s.step(dt)
        _check(o, s, c["W"], f"dt change sigma={sigma}")


def test_finer_checkpoint_loads_into_a_coarser_simulation(tmp_path):
    # created on 36^3, loaded with a 72^3 checkpoint: grid, boxes and occupancy
    # rows follow the checkpoint, and the steps continue exactly
    import paper_1701_06658_amd as gg
    fine = make_config(2, N=72, G=125)
    coarse = make_config(2, N=36, G=125)
    a = _sim(fine)
    a.step(fine["dt"], 2)
    path = str(tmp_path / "fine.ckpt")
    a.save(path)
    b = gg.Simulation(coarse["labels"], coarse["W"], G=fine["G"], precision="fp64")
    b.load(path)
    assert b.n == (72, 72, 72)
    a.step(fine["dt"], 3)
    b.step(fine["dt"], 3)
    _same(a.state(), b.state())
    assert np.array_equal(a.labels(), b.labels())
