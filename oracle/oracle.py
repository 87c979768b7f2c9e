"""ctypes wrapper of the C oracle in ``gg_oracle.c`` (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gg_oracle.c")
_LIB = os.path.join(_HERE, "libgg_oracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


# -O3 for x86-64-v3 (AVX2, which the hosts of MI355X nodes have); products and
# sums are still rounded separately (no contraction), so results do not depend
# on the flags.
ORACLE_CFLAGS = ["-O3", "-march=x86-64-v3", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build_oracle(force=True):
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", *ORACLE_CFLAGS, "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle()
    lib = C.CDLL(_LIB)
    i32_3 = C.POINTER(C.c_int32)
    lib.orc_create.restype = C.c_void_p
    lib.orc_create.argtypes = [C.c_int, _i32p, C.c_double, _i32p, C.c_int32]
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_set_physics.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_void_p,
                                    C.c_double, C.c_double]
    lib.orc_step.argtypes = [C.c_void_p, C.c_double]
    lib.orc_keep_intermediates.argtypes = [C.c_void_p, C.c_int]
    lib.orc_grain_count.argtypes = [C.c_void_p]
    lib.orc_alive_count.argtypes = [C.c_void_p]
    for f in (lib.orc_get_box, lib.orc_get_prev_box):
        f.argtypes = [C.c_void_p, C.c_int, _i32p, _i32p]
    for f in (lib.orc_get_phi, lib.orc_get_psi, lib.orc_get_phic):
        f.argtypes = [C.c_void_p, C.c_int, _f64p, C.c_int64]
    lib.orc_get_iota.argtypes = [C.c_void_p, C.c_int, _i32p, C.c_int64]
    lib.orc_set_grain.argtypes = [C.c_void_p, C.c_int, C.c_int, _i32p, _i32p, C.c_void_p,
                                  C.c_void_p]
    lib.orc_volumes.argtypes = [C.c_void_p, _f64p]
    lib.orc_labels.argtypes = [C.c_void_p, _i32p]
    lib.orc_convolve_box.argtypes = [C.c_int, _i32p, C.c_double, C.c_double, _i32p, _i32p,
                                     _f64p, _f64p]
    lib.orc_redistance_box.argtypes = [C.c_int, _i32p, C.c_double, _i32p, _i32p, _f64p, _f64p]
    lib.orc_redistance_box_euclid.argtypes = [C.c_int, _i32p, C.c_double, _i32p, _i32p, _f64p, _f64p]
    lib.orc_euclid_sweeps.argtypes = [C.c_int, C.c_double]
    lib.orc_set_redistance.argtypes = [C.c_void_p, C.c_int]
    lib.orc_coarsen.argtypes = [C.c_void_p, _i32p]
    lib.orc_grain_areas.argtypes = [C.c_void_p, _f64p, _f64p]
    lib.orc_coarse_sample_box.argtypes = [C.c_int, _i32p, _i32p, C.c_double, _i32p, _i32p, _f64p, _i32p, _i32p,
                                          _f64p]
    lib.orc_misorientation_deg.restype = C.c_double
    lib.orc_misorientation_deg.argtypes = [_f64p, _f64p]
    lib.orc_pair_weight.restype = C.c_double
    lib.orc_pair_weight.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double)]
    lib.orc_set_closest_point.argtypes = [C.c_void_p, C.c_int, C.c_double]
    lib.orc_closest_weights.argtypes = [C.c_void_p, C.c_int, _f64p, C.c_int64]
    lib.orc_closest_box.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_double, _f64p,
                                    np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS"), _i32p]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_num_threads.argtypes = [C.c_int]
    del i32_3
    _lib = lib
    return lib


def _grid(n):
    n = [int(v) for v in n]
    if len(n) == 2:
        n.append(1)
    return np.array(n, dtype=np.int32)


def _shape(ext):
    return (int(ext[2]), int(ext[1]), int(ext[0]))


class Oracle:
    """One oracle simulation built from a label field of shape (nz, ny, nx)."""

    def __init__(self, labels, band, G=None, dim=None):
        lib = load_library()
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        if labels.ndim == 2:
            labels = labels[None]
        nz, ny, nx = labels.shape
        self.dim = int(dim or (2 if nz == 1 else 3))
        self.n = _grid((nx, ny, nz))
        self.G = int(G if G is not None else labels.max() + 1)
        self.band = float(band)
        self._lib = lib
        self._p = lib.orc_create(self.dim, self.n, self.band, labels.ravel(), self.G)
        if not self._p:
            raise ValueError("oracle rejected the inputs")

    def close(self):
        if getattr(self, "_p", None):
            self._lib.orc_destroy(self._p)
            self._p = None

    __del__ = close

    def set_physics(self, mode, quat=None, theta_c_deg=15.0, energy=None, h_phys=0.0,
                    gamma_max=0.0):
        q = None if quat is None else np.ascontiguousarray(quat, dtype=np.float64)
        e = None if energy is None else np.ascontiguousarray(energy, dtype=np.float64)
        rc = self._lib.orc_set_physics(self._p, int(mode),
                                       None if q is None else q.ctypes.data_as(C.c_void_p),
                                       float(theta_c_deg),
                                       None if e is None else e.ctypes.data_as(C.c_void_p),
                                       float(h_phys), float(gamma_max))
        if rc != 0:
            raise ValueError("oracle rejected the physics inputs")
        self._keep_q, self._keep_e = q, e

    def set_closest_point(self, on=True, tube=2.0):
        """Correction weights from the closest grain-boundary point inside the
        tube |phi| < tube (sec. 3.2); needs the misorientation weights."""
        if self._lib.orc_set_closest_point(self._p, int(bool(on)), float(tube)) != 0:
            raise ValueError("bad closest-point arguments")

    def closest_weights(self, k):
        """The correction weight map of grain k for the next step (box shape)."""
        alive, lo, ext = self.box(k)
        if not alive:
            return None
        out = np.empty(int(np.prod(ext)), np.float64)
        if self._lib.orc_closest_weights(self._p, int(k), out, out.size) != 1:
            raise ValueError("closest weights need the misorientation weights")
        return out.reshape(_shape(ext))

    def set_redistance(self, mode):
        """0: the paper's taxicab spreading; 1: Euclidean fast sweeping (steps after this call)."""
        if self._lib.orc_set_redistance(self._p, int(mode)) != 0:
            raise ValueError("unknown re-initialization scheme")

    def coarsen(self, n_new):
        """Project every grain onto the coarser periodic grid n_new (same ratio on every axis)."""
        nn = _grid(n_new)
        if self._lib.orc_coarsen(self._p, nn) != 0:
            raise ValueError("oracle rejected the coarser grid")
        self.n = nn

    def keep_intermediates(self, on=True):
        self._lib.orc_keep_intermediates(self._p, int(bool(on)))

    def step(self, dt, n=1):
        for _ in range(int(n)):
            if self._lib.orc_step(self._p, float(dt)) != 0:
                raise ValueError("oracle step failed")

    def alive_count(self):
        return self._lib.orc_alive_count(self._p)

    def box(self, k, prev=False):
        lo = np.zeros(3, np.int32)
        ext = np.zeros(3, np.int32)
        f = self._lib.orc_get_prev_box if prev else self._lib.orc_get_box
        alive = f(self._p, int(k), lo, ext)
        if alive < 0:
            raise IndexError(k)
        return bool(alive), lo, ext

    def _field(self, getter, k, prev=False):
        alive, lo, ext = self.box(k, prev)
        if not alive:
            return None
        out = np.empty(int(np.prod(ext)), np.float64)
        if getter(self._p, int(k), out, out.size) != 0:
            return None
        return out.reshape(_shape(ext))

    def phi(self, k):
        return self._field(self._lib.orc_get_phi, k)

    def psi(self, k):
        return self._field(self._lib.orc_get_psi, k, prev=True)

    def phic(self, k):
        return self._field(self._lib.orc_get_phic, k, prev=True)

    def iota(self, k):
        alive, lo, ext = self.box(k)
        if not alive:
            return None
        out = np.empty(int(np.prod(ext)), np.int32)
        if self._lib.orc_get_iota(self._p, int(k), out, out.size) != 0:
            return None
        return out.reshape(_shape(ext))

    def set_grain(self, k, alive, lo=None, ext=None, phi=None, iota=None):
        lo = np.ascontiguousarray(lo if lo is not None else [0, 0, 0], dtype=np.int32)
        ext = np.ascontiguousarray(ext if ext is not None else [1, 1, 1], dtype=np.int32)
        ph = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
        io = None if iota is None else np.ascontiguousarray(iota, dtype=np.int32)
        rc = self._lib.orc_set_grain(self._p, int(k), int(bool(alive)), lo, ext,
                                     None if ph is None else ph.ctypes.data_as(C.c_void_p),
                                     None if io is None else io.ctypes.data_as(C.c_void_p))
        if rc != 0:
            raise ValueError("oracle rejected the grain state")

    def volumes(self):
        out = np.zeros(self.G, np.float64)
        self._lib.orc_volumes(self._p, out)
        return out

    def areas(self):
        """(area, weighted): per-grain interface areas and Read-Shockley-weighted areas."""
        a = np.zeros(self.G, np.float64)
        w = np.zeros(self.G, np.float64)
        self._lib.orc_grain_areas(self._p, a, w)
        return a, w

    def labels(self):
        out = np.empty(int(np.prod(self.n)), np.int32)
        self._lib.orc_labels(self._p, out)
        return out.reshape(int(self.n[2]), int(self.n[1]), int(self.n[0]))

    def state(self):
        """All grains: dict with alive (G,), lo (G,3), ext (G,3), phi (list of arrays or None)."""
        alive = np.zeros(self.G, bool)
        lo = np.zeros((self.G, 3), np.int32)
        ext = np.zeros((self.G, 3), np.int32)
        phis = []
        for k in range(self.G):
            a, l, e = self.box(k)
            alive[k] = a
            lo[k] = l
            ext[k] = e
            phis.append(self.phi(k) if a else None)
        return dict(alive=alive, lo=lo, ext=ext, phi=phis)


def convolve_box(f, band, sigma, n, dim=None):
    """Predictor convolution of one box field f (shape (ez, ey, ex)) on grid n."""
    lib = load_library()
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim == 2:
        f = f[None]
    nn = _grid(n)
    dim = dim or (2 if nn[2] == 1 else 3)
    ext = np.array([f.shape[2], f.shape[1], f.shape[0]], np.int32)
    out = np.empty_like(f)
    R = lib.orc_convolve_box(dim, nn, float(band), float(sigma), np.zeros(3, np.int32), ext,
                             f.ravel(), out.ravel())
    if R < 0:
        raise ValueError("bad arguments")
    return out


def redistance_box(f, band, n, dim=None, euclid=False):
    """Re-initialization of one box field f (shape (ez, ey, ex)) on grid n
    (euclid: the Euclidean fast-sweeping scheme instead of the taxicab one)."""
    lib = load_library()
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim == 2:
        f = f[None]
    nn = _grid(n)
    dim = dim or (2 if nn[2] == 1 else 3)
    ext = np.array([f.shape[2], f.shape[1], f.shape[0]], np.int32)
    out = np.empty_like(f)
    fn = lib.orc_redistance_box_euclid if euclid else lib.orc_redistance_box
    if fn(dim, nn, float(band), np.zeros(3, np.int32), ext, f.ravel(), out.ravel()) != 0:
        raise ValueError("bad arguments")
    return out


def closest_box(f, n, tube, dim=None):
    """Closest piece of the linearised zero level set of one box field f (shape
    (ez, ey, ex)) for every voxel with |f| < tube: (d2, cell, piece), d2 = -1
    elsewhere.  A box axis equal to the grid's wraps around."""
    lib = load_library()
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim == 2:
        f = f[None]
    nn = _grid(n)
    dim = dim or (2 if nn[2] == 1 else 3)
    ext = np.array([f.shape[2], f.shape[1], f.shape[0]], np.int32)
    d2 = np.empty(f.shape, np.float64)
    cell = np.empty(f.shape, np.int64)
    piece = np.empty(f.shape, np.int32)
    if lib.orc_closest_box(dim, nn, ext, f.ravel(), float(tube), d2.ravel(), cell.ravel(), piece.ravel()) != 0:
        raise ValueError("bad arguments")
    return d2, cell, piece


def coarse_sample_box(f, band, n, n_new, lo, new_lo, new_ext, dim=None):
    """The coarsening's remap (before re-initialization) of one box field f
    (shape (ez, ey, ex), box origin lo on grid n) at the nodes of the box
    (new_lo, new_ext) of grid n_new."""
    lib = load_library()
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim == 2:
        f = f[None]
    nn, npp = _grid(n), _grid(n_new)
    dim = dim or (2 if nn[2] == 1 else 3)
    ext = np.array([f.shape[2], f.shape[1], f.shape[0]], np.int32)
    ne = np.ascontiguousarray(new_ext, np.int32)
    out = np.empty(_shape(ne), np.float64)
    lib.orc_coarse_sample_box(dim, nn, npp, float(band), np.ascontiguousarray(lo, np.int32), ext, f.ravel(),
                              np.ascontiguousarray(new_lo, np.int32), ne, out.ravel())
    return out


def misorientation_deg(qa, qb):
    lib = load_library()
    return lib.orc_misorientation_deg(np.ascontiguousarray(qa, np.float64),
                                      np.ascontiguousarray(qb, np.float64))


def pair_weight(theta_deg, theta_c_deg=15.0):
    lib = load_library()
    mob = C.c_double(0.0)
    w = lib.orc_pair_weight(float(theta_deg), float(theta_c_deg), C.byref(mob))
    return w, mob.value


def num_threads():
    return load_library().orc_num_threads()


def set_num_threads(n):
    """Threads of the oracle's following calls."""
    load_library().orc_set_num_threads(int(n))


def euclid_sweeps(dim, band):
    """Jacobi sweeps the Euclidean scheme takes (even, >= ceil(sqrt(dim) band) + 1)."""
    return int(load_library().orc_euclid_sweeps(int(dim), float(band)))
