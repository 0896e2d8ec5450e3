"""CPU oracle for the pMSz correction -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It never touches the GPU library, and the GPU
library never touches it.  The arithmetic lives in ``pmsz_oracle.c`` (plain C,
OpenMP across vertices); this module only marshals numpy arrays.

Every function follows a passage of the paper (pMSz, arXiv 2601.01787):
directions = n_min / n_max of Sec. IV-A, flags = the ascending, descending and
FPmax rules of Sec. IV-A / III-B, edit = Eq. 1, labels = integral lines and
segmentations of Sec. III-A, verify = the counts of Sec. V-D.
"""
import ctypes
import os

import numpy as np

from . import build as _build

F32, F64 = 0, 1
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "NONFINITE", 3: "INPUT_BOUND",
          4: "NOT_CONVERGED", 5: "STALLED", 6: "OOM"}

_lib = None


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("steps_applied", ctypes.c_int64),
                ("flagged_final", ctypes.c_int64), ("stalled_flags", ctypes.c_int64),
                ("mismatch_initial", ctypes.c_int64), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class Report(ctypes.Structure):
    _fields_ = [("bound_violations", ctypes.c_int64), ("asc_mismatch", ctypes.c_int64),
                ("desc_mismatch", ctypes.c_int64), ("false_max", ctypes.c_int64),
                ("false_min", ctypes.c_int64), ("missed_max", ctypes.c_int64),
                ("missed_min", ctypes.c_int64), ("wrong_max_label", ctypes.c_int64),
                ("wrong_min_label", ctypes.c_int64), ("wrong_label", ctypes.c_int64),
                ("vertices_edited", ctypes.c_int64), ("max_abs_err", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=True)
        L = ctypes.CDLL(path)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        grid = [i32, i64, i64, i64]
        L.orc_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_xi_t.argtypes = [i32, dbl]
        L.orc_xi_t.restype = dbl
        L.orc_bounds.argtypes = [i32, vp, i64, dbl, vp, vp]
        L.orc_edit.argtypes = [i32, vp, vp, i64, vp]
        L.orc_directions.argtypes = grid + [i32, vp, vp]
        L.orc_directions_at.argtypes = grid + [i32, vp, vp, i64, vp]
        L.orc_validate.argtypes = grid + [i32, vp, vp, dbl]
        L.orc_flags.argtypes = grid + [i32, vp, vp, vp]
        L.orc_flags.restype = i64
        L.orc_correct.argtypes = grid + [i32, vp, vp, dbl, vp, i64, ctypes.POINTER(Stats)]
        L.orc_correct_mode.argtypes = grid + [i32, vp, vp, dbl, vp, i64, i32,
                                              ctypes.POINTER(Stats)]
        L.orc_correct_core.argtypes = grid + [i32, vp, vp, dbl, vp, i64, i32, vp,
                                              ctypes.POINTER(Stats)]
        L.orc_flags_targeted.argtypes = grid + [i32, vp, vp, vp, vp]
        L.orc_flags_targeted.restype = i64
        L.orc_labels.argtypes = grid + [vp, vp, vp]
        L.orc_labels_at.argtypes = grid + [i32, vp, vp, i64, vp, vp]
        L.orc_verify.argtypes = grid + [i32, vp, vp, vp, dbl, ctypes.POINTER(Report)]
        for name in ("orc_directions", "orc_directions_at", "orc_validate", "orc_correct",
                     "orc_correct_mode", "orc_correct_core",
                     "orc_labels", "orc_labels_at", "orc_verify"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _dtype_code(a):
    if a.dtype == np.float32:
        return F32
    if a.dtype == np.float64:
        return F64
    raise TypeError("field must be float32 or float64, got %s" % a.dtype)


def grid_of(a):
    """(ndim, nx, ny, nz) of a C-ordered array shaped (ny, nx) or (nz, ny, nx)."""
    if a.ndim == 2:
        return 2, a.shape[1], a.shape[0], 1
    if a.ndim == 3:
        return 3, a.shape[2], a.shape[1], a.shape[0]
    raise ValueError("field must be 2D (ny, nx) or 3D (nz, ny, nx)")


def _c(a):
    if not (a.flags.c_contiguous and a.flags.aligned):
        raise ValueError("arrays must be C-contiguous")
    return a


def threads():
    return lib().orc_threads()


def set_threads(n):
    lib().orc_set_threads(int(n))


def xi_t(dtype, xi):
    return lib().orc_xi_t(F32 if np.dtype(dtype) == np.float32 else F64, float(xi))


def bounds(f, xi):
    f = _c(np.asarray(f))
    lb = np.empty_like(f)
    ub = np.empty_like(f)
    lib().orc_bounds(_dtype_code(f), _ptr(f), f.size, float(xi), _ptr(lb), _ptr(ub))
    return lb, ub


def edit(g, lb):
    g = _c(np.asarray(g))
    lb = _c(np.asarray(lb, dtype=g.dtype))
    out = np.empty_like(g)
    lib().orc_edit(_dtype_code(g), _ptr(g), _ptr(lb), g.size, _ptr(out))
    return out


def directions(h):
    h = _c(h)
    out = np.empty(h.shape, dtype=np.uint8)
    s = lib().orc_directions(*grid_of(h), _dtype_code(h), _ptr(h), _ptr(out))
    if s:
        raise ValueError(STATUS[s])
    return out


def directions_at(h, idx):
    h = _c(h)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.shape, dtype=np.uint8)
    s = lib().orc_directions_at(*grid_of(h), _dtype_code(h), _ptr(h), _ptr(idx), idx.size,
                                _ptr(out))
    if s:
        raise ValueError(STATUS[s])
    return out


def validate(f, fhat, xi):
    f, fhat = _c(f), _c(fhat)
    return STATUS[lib().orc_validate(*grid_of(f), _dtype_code(f), _ptr(f), _ptr(fhat),
                                     float(xi))]


def flags(g, dirs_f):
    """Flag set of one iteration from g alone; returns (flags uint8, mismatches)."""
    g, dirs_f = _c(g), _c(dirs_f)
    out = np.empty(g.shape, dtype=np.uint8)
    m = lib().orc_flags(*grid_of(g), _dtype_code(g), _ptr(g), _ptr(dirs_f), _ptr(out))
    return out, int(m)


EDIT_MODES = {"halving": 0, "targeted": 1}


def correct(f, fhat, xi, max_iters=1 << 40, dirs_f=None, mode="halving"):
    """Run the correction on a copy of fhat; returns (g, stats dict).
    mode: "halving" (Eq. 1 with half the gap to the bound) or "targeted"
    (each target lowered just below its rival, never below the bound)."""
    f = _c(f)
    g = np.array(fhat, dtype=f.dtype, copy=True, order="C")
    st = Stats()
    lib().orc_correct_mode(*grid_of(f), _dtype_code(f), _ptr(f), _ptr(g), float(xi),
                           _ptr(dirs_f) if dirs_f is not None else None, int(max_iters),
                           EDIT_MODES[mode], ctypes.byref(st))
    d = st.as_dict()
    d["status"] = STATUS[d["status"]]
    return g, d


def correct_core(f, g, xi, core, max_iters=1 << 40, dirs_f=None, mode="halving"):
    """The correction of one block of a decomposed domain (Sec. IV-B), in
    place on g: the loop of `correct`, with only the vertices of the box
    core = (x0, x1, y0, y1, z0, z1) (half-open) compared; flags may target any
    vertex of the array.  Returns the stats dict."""
    f, g = _c(f), _c(g)
    box = (ctypes.c_int64 * 6)(*[int(c) for c in core])
    st = Stats()
    lib().orc_correct_core(*grid_of(f), _dtype_code(f), _ptr(f), _ptr(g), float(xi),
                           _ptr(dirs_f) if dirs_f is not None else None, int(max_iters),
                           EDIT_MODES[mode], ctypes.cast(box, ctypes.c_void_p),
                           ctypes.byref(st))
    d = st.as_dict()
    d["status"] = STATUS[d["status"]]
    return d


def flags_targeted(g, dirs_f):
    """Flag set of one iteration with the targeted proposals: returns
    (flags uint8, proposals float64 (+inf where none), mismatches)."""
    g, dirs_f = _c(g), _c(dirs_f)
    out = np.empty(g.shape, dtype=np.uint8)
    prop = np.empty(g.shape, dtype=np.float64)
    m = lib().orc_flags_targeted(*grid_of(g), _dtype_code(g), _ptr(g), _ptr(dirs_f), _ptr(out),
                                 _ptr(prop))
    return out, prop, int(m)


def labels(dirs):
    dirs = _c(dirs)
    mx = np.empty(dirs.shape, dtype=np.int32)
    mn = np.empty(dirs.shape, dtype=np.int32)
    s = lib().orc_labels(*grid_of(dirs), _ptr(dirs), _ptr(mx), _ptr(mn))
    if s:
        raise ValueError(STATUS[s])
    return mx, mn


def labels_at(h, idx):
    h = _c(h)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    mx = np.empty(idx.shape, dtype=np.int32)
    mn = np.empty(idx.shape, dtype=np.int32)
    s = lib().orc_labels_at(*grid_of(h), _dtype_code(h), _ptr(h), _ptr(idx), idx.size,
                            _ptr(mx), _ptr(mn))
    if s:
        raise ValueError(STATUS[s])
    return mx, mn


def verify(f, g, fhat, xi):
    f, g = _c(f), _c(g)
    if fhat is not None:
        fhat = _c(fhat)
    r = Report()
    s = lib().orc_verify(*grid_of(f), _dtype_code(f), _ptr(f), _ptr(g), _ptr(fhat),
                         float(xi), ctypes.byref(r))
    if s:
        raise ValueError(STATUS[s])
    return r.as_dict()
