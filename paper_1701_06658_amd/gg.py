"""ctypes binding of the C ABI in include/gg.h (argument marshalling only).

Every step of the method runs in the HIP library ``libgg.so``; this module only
converts arguments.  It raises if the library has not been built: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgg.so")

GG_FP64, GG_FP32 = 0, 1
PHYS_NONE, PHYS_MISORIENTATION, PHYS_BULK = 0, 1, 2
GG_REDIST_TAXICAB, GG_REDIST_EUCLID = 0, 1

STATUS = {0: "GG_OK", 1: "GG_E_ARG", 2: "GG_E_NOMEM", 3: "GG_E_HIP", 4: "GG_E_CAPACITY",
          5: "GG_E_SMALLBUF", 6: "GG_E_NUMERIC", 7: "GG_E_POISONED", 8: "GG_E_UNSUPPORTED",
          9: "GG_E_NODEVICE"}

EXPORTS = ["gg_create", "gg_step", "gg_sync", "gg_grain_count", "gg_grain_volumes", "gg_labels",
           "gg_stats", "gg_get_boxes", "gg_get_values", "gg_get_iota", "gg_load_state",
           "gg_keep_intermediates", "gg_get_intermediate", "gg_status_str", "gg_last_error",
           "gg_destroy", "gg_version", "gg_profile", "gg_get_kernel_times", "gg_coarsen", "gg_grain_areas",
           "gg_grain_sdf", "gg_save", "gg_load", "gg_autotune", "gg_grain_areas_noalloc"]

KERNEL_CLASSES = ["predict", "compare", "reinit", "reinit_sweep", "plan", "closest"]
FLAG_ORDER_ID = 1
FLAG_CLOSEST_POINT = 2


class GGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("band", C.c_double),
                ("precision", C.c_int32), ("physics", C.c_int32), ("theta_c_deg", C.c_double),
                ("voxel_m", C.c_double), ("gamma_max", C.c_double),
                ("capacity_headroom", C.c_double), ("redistance", C.c_int32),
                ("batched", C.c_int32), ("flags", C.c_uint32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


def torch_allocator():
    """A gg_allocator over PyTorch's caching allocator (the blocks show up in
    torch.cuda.memory_allocated and are reused by torch after gg_destroy)."""
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except RuntimeError:
            return None

    def _free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    a = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    a._keep = (_alloc, _free)
    return a


class KernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 6), ("launches", C.c_int64 * 6), ("voxels", C.c_int64 * 6)]


class Tuning(C.Structure):
    _fields_ = [("order_size", C.c_int32), ("lds_bytes", C.c_int32), ("small_bytes", C.c_int32),
                ("candidates", C.c_int32), ("ns_per_gv", C.c_double * 8), ("cand_order", C.c_int32 * 8),
                ("cand_lds", C.c_int32 * 8), ("cand_small", C.c_int32 * 8)]


class StepStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("total_grain_voxels", C.c_int64), ("alive", C.c_int32),
                ("kernel_radius", C.c_int32),
                ("grain_voxels", C.c_int64), ("capacity", C.c_int64),
                ("superposition", C.c_double), ("last_step_ms", C.c_double), ("n", C.c_int32 * 3),
                ("dim", C.c_int32)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libgg.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1701_06658_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "gg_create": (i32, [C.POINTER(Config), vp, i32, vp, vp, vp, C.POINTER(Allocator), C.POINTER(vp)]),
        "gg_step": (i32, [vp, dbl, i32]),
        "gg_sync": (i32, [vp]),
        "gg_grain_count": (i32, [vp, C.POINTER(i32)]),
        "gg_grain_volumes": (i32, [vp, vp, i64]),
        "gg_labels": (i32, [vp, vp, i64, i32]),
        "gg_stats": (i32, [vp, C.POINTER(StepStats)]),
        "gg_get_boxes": (i32, [vp, vp, vp, vp, vp, i64]),
        "gg_get_values": (i32, [vp, vp, i64]),
        "gg_get_iota": (i32, [vp, vp, i64]),
        "gg_load_state": (i32, [vp, vp, vp, vp, vp, vp]),
        "gg_coarsen": (i32, [vp, vp]),
        "gg_grain_areas": (i32, [vp, vp, vp, i64]),
        "gg_grain_areas_noalloc": (i32, [vp, vp, vp, i64]),
        "gg_grain_sdf": (i32, [vp, i32, vp, vp, vp, i64]),
        "gg_autotune": (i32, [vp, dbl, i32, C.POINTER(Tuning)]),
        "gg_save": (i32, [vp, C.c_char_p]),
        "gg_load": (i32, [vp, C.c_char_p]),
        "gg_keep_intermediates": (i32, [vp, i32]),
        "gg_get_intermediate": (i32, [vp, i32, vp, i64, vp, vp, vp, vp, i64]),
        "gg_status_str": (C.c_char_p, [i32]),
        "gg_last_error": (C.c_char_p, [vp]),
        "gg_destroy": (None, [vp]),
        "gg_version": (C.c_char_p, []),
        "gg_profile": (i32, [vp, i32]),
        "gg_get_kernel_times": (i32, [vp, C.POINTER(KernelTimes)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class Simulation:
    """One grain-growth simulation on the GPU, created from a label field.

    labels: int array (nz, ny, nx) (nz == 1 in 2D), values in [0, G).
    precision: "fp64" (plain) or "fp32" (mixed).
    stream: optional hipStream_t handle (int), e.g. torch.cuda.current_stream().cuda_stream.
    allocator: None (the library's hipMalloc), "torch" (PyTorch's caching
    allocator, on `stream` or torch's current stream) or an Allocator.
    batched: gg_step queues captured HIP graphs and returns without waiting.
    order_size: per-grain kernels take the largest boxes first (False: grain-id order).
    closest_point: correction weights from the closest grain-boundary point in
    the tube |phi| < 2 (needs physics with the misorientation weights).
    """

    def __init__(self, labels, band, G=None, precision="fp64", physics=0, quat=None,
                 theta_c_deg=15.0, energy=None, voxel_m=0.0, gamma_max=0.0, stream=None,
                 headroom=0.0, redistance="taxicab", allocator=None, batched=False, order_size=True,
                 closest_point=False):
        lib = load_library()
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        if labels.ndim == 2:
            labels = labels[None]
        nz, ny, nx = labels.shape
        self.dim = 2 if nz == 1 else 3
        self.n = (nx, ny, nz)
        self.G = int(G if G is not None else labels.max() + 1)
        cfg = Config()
        cfg.dim = self.dim
        cfg.n[0], cfg.n[1], cfg.n[2] = nx, ny, nz
        cfg.band = float(band)
        cfg.precision = {"fp64": GG_FP64, "fp32": GG_FP32}[precision]
        cfg.physics = int(physics)
        cfg.theta_c_deg = float(theta_c_deg)
        cfg.voxel_m = float(voxel_m)
        cfg.gamma_max = float(gamma_max)
        cfg.capacity_headroom = float(headroom)
        cfg.redistance = {"taxicab": GG_REDIST_TAXICAB, "euclid": GG_REDIST_EUCLID}[redistance]
        cfg.batched = 1 if batched else 0
        cfg.flags = (0 if order_size else FLAG_ORDER_ID) | (FLAG_CLOSEST_POINT if closest_point else 0)
        q = None if quat is None else np.ascontiguousarray(quat, dtype=np.float64)
        e = None if energy is None else np.ascontiguousarray(energy, dtype=np.float64)
        if allocator == "torch":
            import torch
            allocator = torch_allocator()
            if not stream:
                stream = torch.cuda.current_stream().cuda_stream
        self._allocator = allocator  # the callbacks must outlive the simulation
        h = C.c_void_p()
        st = lib.gg_create(C.byref(cfg), _ptr(labels), self.G, _ptr(q), _ptr(e),
                           C.c_void_p(int(stream)) if stream else None,
                           C.byref(allocator) if allocator is not None else None, C.byref(h))
        if st != 0:
            raise GGError(st, lib.gg_last_error(None).decode())
        self._lib = lib
        self._h = h
        self.precision = precision
        self.band = float(band)

    def _check(self, st):
        if st != 0:
            raise GGError(st, self._lib.gg_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gg_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, dt, n=1):
        self._check(self._lib.gg_step(self._h, float(dt), int(n)))

    def sync(self):
        self._check(self._lib.gg_sync(self._h))

    def grain_sdf(self, k):
        """(lo, ext, values (ez, ey, ex)) of grain k, or None if it is extinct."""
        lo = np.zeros(3, np.int32)
        ext = np.zeros(3, np.int32)
        self._check(self._lib.gg_grain_sdf(self._h, int(k), _ptr(lo), _ptr(ext), None, 0))
        if not ext.any():
            return None
        out = np.empty(int(np.prod(ext)), np.float64)
        self._check(self._lib.gg_grain_sdf(self._h, int(k), _ptr(lo), _ptr(ext), _ptr(out), out.size))
        return lo, ext, out.reshape(int(ext[2]), int(ext[1]), int(ext[0]))

    def autotune(self, dt, steps_per_candidate=1):
        """Pick the launch schedule with the fastest steps (advances the
        simulation).  Returns a dict: the chosen order_size, lds_bytes,
        small_bytes and every candidate's device ns per grain voxel."""
        t = Tuning()
        self._check(self._lib.gg_autotune(self._h, float(dt), int(steps_per_candidate), C.byref(t)))
        n = t.candidates
        return dict(order_size=t.order_size, lds_bytes=t.lds_bytes, small_bytes=t.small_bytes,
                    candidates=[dict(order_size=t.cand_order[i], lds_bytes=t.cand_lds[i],
                                     small_bytes=t.cand_small[i], ns_per_gv=t.ns_per_gv[i]) for i in range(n)])

    def save(self, path):
        """Write a checkpoint of the state to `path`."""
        self._check(self._lib.gg_save(self._h, os.fsencode(path)))

    def load(self, path):
        """Replace the state by the checkpoint at `path` (same configuration)."""
        self._check(self._lib.gg_load(self._h, os.fsencode(path)))
        self.n = tuple(int(v) for v in self.stats()["n"])

    def areas(self):
        """(area, weighted): per-grain interface areas and Read-Shockley-weighted areas (FP64)."""
        a = np.zeros(self.G, np.float64)
        w = np.zeros(self.G, np.float64)
        self._check(self._lib.gg_grain_areas(self._h, _ptr(a), _ptr(w), self.G))
        return a, w

    def areas_noalloc(self, area_dev, weighted_dev=None):
        """gg_grain_areas_noalloc: the areas written into device buffers (objects
        with data_ptr() and numel(), e.g. torch tensors of float64 on the
        simulation's device); stream-ordered, the call does not wait."""
        cap = area_dev.numel() if weighted_dev is None else min(area_dev.numel(), weighted_dev.numel())
        self._check(self._lib.gg_grain_areas_noalloc(
            self._h, C.c_void_p(area_dev.data_ptr()),
            C.c_void_p(weighted_dev.data_ptr()) if weighted_dev is not None else None, cap))

    def coarsen(self, n_new):
        """Project the state onto the coarser periodic grid n_new = (nx, ny, nz) (nz = 1 in 2D)."""
        nn = np.ascontiguousarray([int(v) for v in n_new] + [1] * (3 - len(n_new)), dtype=np.int32)
        self._check(self._lib.gg_coarsen(self._h, _ptr(nn)))
        self.n = (int(nn[0]), int(nn[1]), int(nn[2]))

    def alive_count(self):
        v = C.c_int32()
        self._check(self._lib.gg_grain_count(self._h, C.byref(v)))
        return v.value

    def volumes(self):
        out = np.zeros(self.G, np.float64)
        self._check(self._lib.gg_grain_volumes(self._h, _ptr(out), out.size))
        return out

    def labels(self, device_out=None):
        """Voxel labels as a numpy array, or written into a device buffer (torch tensor)."""
        if device_out is not None:
            self._check(self._lib.gg_labels(self._h, C.c_void_p(device_out.data_ptr()),
                                            device_out.numel(), 1))
            return device_out
        out = np.empty(int(np.prod(self.n)), np.int32)
        self._check(self._lib.gg_labels(self._h, _ptr(out), out.size, 0))
        return out.reshape(self.n[2], self.n[1], self.n[0])

    def stats(self):
        s = StepStats()
        self._check(self._lib.gg_stats(self._h, C.byref(s)))
        out = {f: getattr(s, f) for f, _ in StepStats._fields_}
        out["n"] = tuple(out["n"])
        return out

    def profile(self, on=True):
        """Per-kernel HIP-event timing on the simulation's stream (resets the sums)."""
        self._check(self._lib.gg_profile(self._h, int(bool(on))))

    def kernel_times(self):
        t = KernelTimes()
        self._check(self._lib.gg_get_kernel_times(self._h, C.byref(t)))
        return {name: dict(ms=t.ms[i], launches=t.launches[i], voxels=t.voxels[i])
                for i, name in enumerate(KERNEL_CLASSES) if name != "unused"}

    def boxes(self):
        lo = np.zeros((self.G, 3), np.int32)
        ext = np.zeros((self.G, 3), np.int32)
        alive = np.zeros(self.G, np.int32)
        off = np.zeros(self.G, np.int64)
        self._check(self._lib.gg_get_boxes(self._h, _ptr(lo), _ptr(ext), _ptr(alive), _ptr(off),
                                           self.G))
        return dict(lo=lo, ext=ext, alive=alive.astype(bool), offset=off)

    def values(self):
        b = self.boxes()
        m = int(sum(int(np.prod(e)) for e, a in zip(b["ext"], b["alive"]) if a))
        out = np.empty(max(m, 1), np.float64)
        self._check(self._lib.gg_get_values(self._h, _ptr(out), out.size))
        return b, out[:m]

    def iota(self):
        b = self.boxes()
        m = int(sum(int(np.prod(e)) for e, a in zip(b["ext"], b["alive"]) if a))
        out = np.empty(max(m, 1), np.int32)
        self._check(self._lib.gg_get_iota(self._h, _ptr(out), out.size))
        return b, out[:m]

    def closest_weights(self):
        """Correction weights of the next predictor (closest_point mode): per-grain
        dict like state(), the weights in place of phi."""
        return self.intermediate(2)

    def state(self):
        """Per-grain dict like the oracle's: alive, lo, ext, phi (list of (ez, ey, ex) arrays)."""
        b, v = self.values()
        return _unpack(b, v)

    def load_state(self, alive, lo, ext, phis, iotas=None):
        """Replace the state; phis/iotas: lists of (ez, ey, ex) arrays (None for extinct)."""
        alive = np.ascontiguousarray(alive, dtype=np.uint8)
        lo = np.ascontiguousarray(lo, dtype=np.int32)
        ext = np.ascontiguousarray(ext, dtype=np.int32)
        vals = [np.asarray(p, np.float64).ravel() for p, a in zip(phis, alive) if a]
        flat = np.ascontiguousarray(np.concatenate(vals) if vals else np.zeros(1))
        io = None
        if iotas is not None:
            iv = [np.asarray(p, np.int32).ravel() for p, a in zip(iotas, alive) if a]
            io = np.ascontiguousarray(np.concatenate(iv) if iv else np.zeros(1, np.int32))
        self._check(self._lib.gg_load_state(self._h, _ptr(lo), _ptr(ext), _ptr(alive),
                                            _ptr(flat), _ptr(io)))

    def keep_intermediates(self, on=True):
        self._check(self._lib.gg_keep_intermediates(self._h, int(bool(on))))

    def intermediate(self, which):
        """which 0: predictor output, 1: corrector output, on the step's starting
        boxes; 2: the closest-point correction weights of the next predictor, on
        the current boxes."""
        lo = np.zeros((self.G, 3), np.int32)
        ext = np.zeros((self.G, 3), np.int32)
        alive = np.zeros(self.G, np.int32)
        off = np.zeros(self.G, np.int64)
        cap = 1
        while True:
            out = np.empty(cap, np.float64)
            st = self._lib.gg_get_intermediate(self._h, int(which), _ptr(out), cap, _ptr(lo),
                                               _ptr(ext), _ptr(alive), _ptr(off), self.G)
            if st == 5 and cap == 1:
                m = int(sum(int(np.prod(e)) for e, a in zip(ext, alive) if a))
                msg = self._lib.gg_last_error(self._h).decode()
                cap = int(msg.split("(")[-1].rstrip(")")) if "(" in msg else max(m, 1)
                continue
            self._check(st)
            break
        b = dict(lo=lo, ext=ext, alive=alive.astype(bool), offset=off)
        m = int(sum(int(np.prod(e)) for e, a in zip(ext, alive) if a))
        return _unpack(b, out[:m])


def _unpack(b, v):
    phis = []
    for k in range(len(b["alive"])):
        if not b["alive"][k]:
            phis.append(None)
            continue
        e = b["ext"][k]
        m = int(np.prod(e))
        o = int(b["offset"][k])
        phis.append(v[o:o + m].reshape(int(e[2]), int(e[1]), int(e[0])))
    return dict(alive=np.asarray(b["alive"], bool), lo=b["lo"], ext=b["ext"], phi=phis)


def version():
    return load_library().gg_version().decode()
