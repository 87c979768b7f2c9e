"""Checkpoint / resume, the per-grain state query and the caller's allocator,
on the GPU through the C ABI.

* gg_save then gg_load into a fresh simulation: the following steps are
  bit-identical to the uninterrupted run (FP32 and FP64, with the ID-field of
  the bulk term, with the Euclidean variant, and across a coarsened grid);
  mismatched configurations, corrupt and missing files are rejected and leave
  the simulation unchanged;
* gg_grain_sdf returns a grain's box and values as in the whole-state download, and
  gg_labels writes the same ids into device memory as into host memory;
* a simulation on the caller's allocator runs bit-identically to one on the
  library's own hipMalloc, and every block goes back to the caller.
"""
import os

import numpy as np
import pytest

from synth import config_dt, make_config
from test_gpu_parity import _physics_inputs

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert np.array_equal(a["alive"], b["alive"])
    assert np.array_equal(a["lo"], b["lo"]) and np.array_equal(a["ext"], b["ext"])
    for pa, pb in zip(a["phi"], b["phi"]):
        assert (pa is None) == (pb is None)
        if pa is not None:
            assert np.array_equal(pa, pb)


def _sim(labels, W, G, precision, **kw):
    import paper_1701_06658_amd as gg
    return gg.Simulation(labels, W, G=G, precision=precision, **kw)


@pytest.mark.parametrize("precision,kind", [("fp32", "plain"), ("fp64", "plain"), ("fp32", "bulk"),
                                            ("fp64", "euclid"), ("fp32", "coarsened")])
def test_checkpoint_resume_is_exact(tmp_path, precision, kind):
    kw = {}
    if kind == "bulk":
        labels, kw, _ = _physics_inputs("bulk")
        G, W, N, sigma = int(labels.max()) + 1, 8.0, 64, 2.0
    else:
        c = make_config(2, N=64, G=125)
        labels, G, W, N, sigma = c["labels"], c["G"], c["W"], 64, c["sigma"]
        if kind == "euclid":
            kw = dict(redistance="euclid")
    dt = config_dt(sigma, N)
    a = _sim(labels, W, G, precision, **kw)
    a.step(dt, 2)
    if kind == "coarsened":
        a.coarsen((48, 48, 48))
        dt = config_dt(sigma, 48)
        a.step(dt)
    path = str(tmp_path / "state.ggc")
    a.save(path)
    a.step(dt, 3)
    b = _sim(labels, W, G, precision, **kw)
    b.load(path)
    assert b.n == a.n and b.stats()["steps"] == a.stats()["steps"] - 3
    b.step(dt, 3)
    _same(a.state(), b.state())
    assert np.array_equal(a.volumes(), b.volumes())
    if kind == "bulk":
        assert np.array_equal(a.iota()[1], b.iota()[1])
    assert os.path.getsize(path) > 0


def test_checkpoint_rejections(tmp_path):
    import paper_1701_06658_amd as gg
    c = make_config(1)
    a = _sim(c["labels"], c["W"], c["G"], "fp64")
    a.step(c["dt"], 2)
    path = str(tmp_path / "a.ggc")
    a.save(path)
    before = a.state()
    other = _sim(c["labels"], c["W"], c["G"], "fp32")
    with pytest.raises(gg.GGError, match="GG_E_ARG"):
        other.load(path)                      # another precision
    bad = tmp_path / "bad.ggc"
    bad.write_bytes(open(path, "rb").read()[:200])
    with pytest.raises(gg.GGError, match="GG_E_ARG"):
        a.load(str(bad))                      # truncated
    with pytest.raises(gg.GGError, match="GG_E_ARG"):
        a.load(str(tmp_path / "missing.ggc"))
    _same(before, a.state())                  # nothing changed
    a.step(c["dt"])                           # and it still steps


def test_grain_sdf_matches_state():
    c = make_config(1)
    s = _sim(c["labels"], c["W"], c["G"], "fp32")
    s.step(c["dt"], 5)
    st = s.state()
    for k in range(c["G"]):
        got = s.grain_sdf(k)
        if not st["alive"][k]:
            assert got is None
            continue
        lo, ext, phi = got
        assert np.array_equal(lo, st["lo"][k]) and np.array_equal(ext, st["ext"][k])
        assert np.array_equal(phi, st["phi"][k])


class _CountingAllocator:
    """A gg_allocator over hipMalloc / hipFree (through ctypes) that counts the
    bytes it has handed out and not yet taken back."""

    def __init__(self, fail_after=None):
        import ctypes as C
        from paper_1701_06658_amd import gg
        hip = C.CDLL("libamdhip64.so")
        hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        hip.hipFree.argtypes = [C.c_void_p]
        self.live, self.calls, self.sizes = 0, 0, {}
        self.dry = False                 # set to refuse every later request

        def _alloc(nbytes, stream, user):
            if self.dry or (fail_after is not None and self.calls >= fail_after):
                return None
            p = C.c_void_p()
            if hip.hipMalloc(C.byref(p), nbytes) != 0:
                return None
            self.sizes[p.value] = nbytes
            self.live += nbytes
            self.calls += 1
            return p.value

        def _free(ptr, stream, user):
            self.live -= self.sizes.pop(ptr)
            hip.hipFree(ptr)

        self._fns = (gg.ALLOC_FN(_alloc), gg.FREE_FN(_free))
        self.struct = gg.Allocator(self._fns[0], self._fns[1], None)


def test_caller_allocator_runs_identically():
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    hip.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
    stream = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(stream)) == 0
    c = make_config(2, N=64, G=125)
    al = _CountingAllocator()
    a = _sim(c["labels"], c["W"], c["G"], "fp64", allocator=al.struct, stream=stream.value)
    b = _sim(c["labels"], c["W"], c["G"], "fp64")
    a.step(c["dt"], 3)
    b.step(c["dt"], 3)
    _same(a.state(), b.state())
    assert al.calls > 10 and al.live > 10 * 2 ** 20      # the arenas came from the caller
    a.close()
    assert al.live == 0 and not al.sizes                   # and all went back


def test_caller_allocator_failure_is_reported():
    # an allocator that runs dry part way through gg_create: GG_E_NOMEM, and
    # every block it did hand out comes back
    import ctypes as C
    import paper_1701_06658_amd as gg
    hip = C.CDLL("libamdhip64.so")
    hip.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
    stream = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(stream)) == 0
    c = make_config(1)
    al = _CountingAllocator(fail_after=12)
    with pytest.raises(gg.GGError, match="GG_E_NOMEM"):
        _sim(c["labels"], c["W"], c["G"], "fp64", allocator=al.struct, stream=stream.value)
    assert al.calls == 12 and al.live == 0


def test_failure_part_way_poisons():
    # a state-changing call whose allocation fails after its argument checks
    # (here gg_coarsen) may leave the state part way replaced: GG_E_NOMEM, then
    # GG_E_POISONED for every later call; gg_destroy still returns every block
    import ctypes as C
    import paper_1701_06658_amd as gg
    hip = C.CDLL("libamdhip64.so")
    hip.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
    stream = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(stream)) == 0
    c = make_config(1)
    al = _CountingAllocator()
    s = _sim(c["labels"], c["W"], c["G"], "fp64", allocator=al.struct, stream=stream.value)
    s.step(c["dt"], 2)
    al.dry = True
    with pytest.raises(gg.GGError, match="GG_E_NOMEM"):
        s.coarsen((32, 32, 1))
    for call in (lambda: s.step(c["dt"]), lambda: s.volumes(), lambda: s.coarsen((32, 32, 1))):
        with pytest.raises(gg.GGError, match="GG_E_POISONED"):
            call()
    s.close()
    assert al.live == 0 and not al.sizes


def test_labels_into_device_memory():
    # gg_labels with a device pointer: stream-ordered write, same ids as the host copy
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    c = make_config(2, N=64, G=125)
    s = _sim(c["labels"], c["W"], c["G"], "fp32")
    s.step(c["dt"], 2)
    n = int(np.prod(s.n))
    buf = C.c_void_p()
    assert hip.hipMalloc(C.byref(buf), 4 * n) == 0

    class _Dev:                      # the two methods the binding reads from a device tensor
        def data_ptr(self):
            return buf.value

        def numel(self):
            return n

    try:
        s.labels(device_out=_Dev())
        s.sync()
        host = np.empty(n, np.int32)
        assert hip.hipMemcpy(host.ctypes.data, buf, 4 * n, 2) == 0   # device to host
        assert np.array_equal(host.reshape(s.n[2], s.n[1], s.n[0]), s.labels())
    finally:
        hip.hipFree(buf)
