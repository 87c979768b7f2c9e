"""gg_grain_areas_noalloc (through the C ABI): interface areas written into
device memory, with the partial sums in the library's static scratch array,
equal those of gg_grain_areas (same kernels, same summation order) on two calls
in a row, the second on a smaller simulation (fewer grains and voxels than the
first, whose partials the scratch still holds); a queued step that must be
taken again with larger buffers is reported, left queued, and taken by gg_sync;
a simulation with more grains than the scratch holds is refused."""
import ctypes as C

import numpy as np
import pytest

from synth import config_dt, make_config
from test_gpu_batched import growing_disk
from test_gpu_parity import _physics_inputs

pytestmark = pytest.mark.gpu


def _hip():
    hip = C.CDLL("libamdhip64.so")
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return hip


class _Dev:
    """The two methods the binding reads from a device buffer."""

    def __init__(self, ptr, n):
        self.ptr, self.n = ptr, n

    def data_ptr(self):
        return self.ptr

    def numel(self):
        return self.n


def _noalloc(s, weighted=True):
    """Areas from gg_grain_areas_noalloc into fresh device buffers (NaN-filled
    first, so an entry the call does not write shows)."""
    hip = _hip()
    G = s.G
    bufs = [C.c_void_p(), C.c_void_p()]
    for b in bufs:
        assert hip.hipMalloc(C.byref(b), 8 * G) == 0
    try:
        nan = np.full(G, np.nan)
        for b in bufs:
            assert hip.hipMemcpy(b, nan.ctypes.data, 8 * G, 1) == 0      # host to device
        s.areas_noalloc(_Dev(bufs[0].value, G), _Dev(bufs[1].value, G) if weighted else None)
        s.sync()
        a, w = np.empty(G), np.empty(G)
        assert hip.hipMemcpy(a.ctypes.data, bufs[0], 8 * G, 2) == 0      # device to host
        assert hip.hipMemcpy(w.ctypes.data, bufs[1], 8 * G, 2) == 0
    finally:
        for b in bufs:
            hip.hipFree(b)
    return a, w


def test_noalloc_equals_areas_two_calls_second_smaller():
    import paper_1701_06658_amd as gg
    # first call: 3D misorientation workload (200 grains, 64^3), FP64, batched
    # steps still queued when the call comes
    labels, gphys, _ = _physics_inputs("misorientation")
    G = int(labels.max()) + 1
    a = gg.Simulation(labels, 8.0, G=G, precision="fp64", batched=True, **gphys)
    a.step(config_dt(2.0, labels.shape[0]), 3)
    na, nw = _noalloc(a)
    ra, rw = a.areas()
    print(f"[noalloc 3d fp64 G={G}] total area {ra.sum():.3f}, weighted {rw.sum():.3f}", flush=True)
    assert np.array_equal(na, ra) and np.array_equal(nw, rw)
    assert not np.array_equal(ra, rw)           # the weights are in play
    # second call: a smaller simulation (2D, 20 grains, FP32), weighted NULL
    c = make_config(1)
    b = gg.Simulation(c["labels"], c["W"], G=c["G"], precision="fp32")
    b.step(c["dt"], 4)
    nb, wb = _noalloc(b, weighted=False)
    rb, _ = b.areas()
    print(f"[noalloc 2d fp32 G={c['G']}] total area {rb.sum():.3f}", flush=True)
    assert np.array_equal(nb, rb)
    assert np.all(np.isnan(wb))                 # weighted_dev NULL: nothing written there
    # and the first simulation again, after the smaller one used the scratch
    na2, nw2 = _noalloc(a)
    assert np.array_equal(na2, ra) and np.array_equal(nw2, rw)


def test_noalloc_leaves_a_failed_batch_queued():
    # exact buffers and a disk grain pushed outward by the bulk term: a queued
    # step's layout outgrows the buffers and fails its capacity check; the
    # no-alloc call reports it and writes nothing, gg_sync takes the steps
    # again, and the call then gives the areas of the completed steps
    import paper_1701_06658_amd as gg
    labels, gphys, _, dt = growing_disk(2)
    s = gg.Simulation(labels, 6.0, G=2, precision="fp64", batched=True, headroom=1.0, **gphys)
    p = gg.Simulation(labels, 6.0, G=2, precision="fp64", **gphys)
    s.step(dt, 6)
    p.step(dt, 6)
    with pytest.raises(gg.GGError, match="GG_E_CAPACITY"):
        _noalloc(s)
    s.sync()
    assert s.stats()["steps"] == 6
    ns, ws = _noalloc(s)
    rp, wp = p.areas()
    assert np.array_equal(ns, rp) and np.array_equal(ws, wp)


def test_noalloc_refuses_more_grains_than_the_scratch():
    import paper_1701_06658_amd as gg
    c = make_config(1)                          # 2D, 64^2, 20 grains
    s = gg.Simulation(c["labels"], c["W"], G=70000, precision="fp32")   # ids 20.. unused
    with pytest.raises(gg.GGError, match="GG_E_CAPACITY"):
        _noalloc(s)
    a, _ = s.areas()                            # the allocating call still serves it
    assert a.shape == (70000,) and np.all(a[c["G"]:] == 0) and a[:c["G"]].sum() > 0
