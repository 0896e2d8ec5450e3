"""pMSz on MI355X: Python binding of libpmsz (gfx950 HIP kernels behind a C ABI).

Argument marshalling only: every step of the correction runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.  There is
no CPU fallback: if ``libpmsz.so`` is missing or fails to load, every call
raises.

Names follow the paper (pMSz, arXiv 2601.01787): ``directions`` computes
n_max / n_min (Sec. IV-A), ``correct`` runs the decrease-only edit loop
(Eq. 1, Sec. IV-A rules), ``labels`` the ascending / descending segmentations
(Sec. III-A), ``verify`` the evaluation counts of Sec. V-D.
"""
import atexit
import ctypes
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmsz.so")

F32, F64 = 0, 1
WS_CORRECT, WS_VERIFY, WS_LABELS, WS_CORRECT_TARGETED = 0, 1, 2, 3
EDIT_MODES = {"halving": 0, "targeted": 1}
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "NONFINITE", 3: "INPUT_BOUND", 4: "NOT_CONVERGED",
          5: "STALLED", 6: "OOM", 7: "DEVICE"}
DEFAULT_MAX_ITERS = 1 << 40
# size of the static device scratch behind pmsz_correct_noalloc
NOALLOC_SCRATCH_BYTES = 32 << 20
STEP_STOP_ON_DONE = 1

# the last two return strings, the others a status code
EXPORTS = ("pmsz_workspace_size", "pmsz_directions", "pmsz_correct",
           "pmsz_batched_workspace_size", "pmsz_correct_batched", "pmsz_labels",
           "pmsz_correct_mode", "pmsz_verify", "pmsz_last_timing", "pmsz_last_rounds",
           "pmsz_session_workspace_size", "pmsz_field_workspace_size", "pmsz_session_create",
           "pmsz_session_add", "pmsz_session_step", "pmsz_session_sync", "pmsz_session_result",
           "pmsz_session_remove", "pmsz_session_destroy", "pmsz_session_step_ex",
           "pmsz_session_request_stop", "pmsz_session_request_stop_when_done",
           "pmsz_session_query", "pmsz_session_finished",
           "pmsz_edits_workspace_size",
           "pmsz_edits_max_bytes", "pmsz_encode_edits", "pmsz_decode_edits",
           "pmsz_blocks_workspace_size", "pmsz_correct_blocks", "pmsz_set_tiles_target",
           "pmsz_get_tiles_target", "pmsz_tune_workspace_size", "pmsz_tune_tiles",
           "pmsz_last_labels", "pmsz_release", "pmsz_correct_noalloc", "pmsz_probe_read",
           "pmsz_status_string", "pmsz_last_error")


class PmszError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("steps_applied", ctypes.c_int64),
                ("flagged_final", ctypes.c_int64), ("stalled_flags", ctypes.c_int64),
                ("mismatch_initial", ctypes.c_int64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["status"] = STATUS.get(d["status"], d["status"])
        return d


class Report(ctypes.Structure):
    _fields_ = [("bound_violations", ctypes.c_int64), ("asc_mismatch", ctypes.c_int64),
                ("desc_mismatch", ctypes.c_int64), ("false_max", ctypes.c_int64),
                ("false_min", ctypes.c_int64), ("missed_max", ctypes.c_int64),
                ("missed_min", ctypes.c_int64), ("wrong_max_label", ctypes.c_int64),
                ("wrong_min_label", ctypes.c_int64), ("wrong_label", ctypes.c_int64),
                ("vertices_edited", ctypes.c_int64), ("max_abs_err", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("engine_ms", ctypes.c_double), ("rounds", ctypes.c_int64),
                ("swept", ctypes.c_int64), ("edits", ctypes.c_int64), ("voxels", ctypes.c_int64),
                ("tiles", ctypes.c_int64), ("grid", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("first_round_ms", ctypes.c_double), ("detect_ms", ctypes.c_double),
                ("apply_ms", ctypes.c_double), ("dirs_ms", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("tail_rounds", ctypes.c_int32),
                ("handbacks", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Round(ctypes.Structure):
    _fields_ = [("detect_ms", ctypes.c_double), ("apply_ms", ctypes.c_double),
                ("swept", ctypes.c_int64), ("flagged", ctypes.c_int64), ("edits", ctypes.c_int64),
                ("sparse", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LabelsInfo(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_int64), ("passes_max", ctypes.c_int64),
                ("passes_min", ctypes.c_int64), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BlocksStats(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_int64), ("local_rounds", ctypes.c_int64),
                ("critical_rounds", ctypes.c_int64), ("lowered", ctypes.c_int64),
                ("steps_applied", ctypes.c_int64), ("compute_ms", ctypes.c_double),
                ("exchange_ms", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["status"] = STATUS.get(d["status"], d["status"])
        return d


class Field(ctypes.Structure):
    _fields_ = [("grid", Grid), ("f", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("xi", ctypes.c_double)]


_lib = None


def load():
    """Load libpmsz.so (built by ``build.py``); raises if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpmsz.so is not built (run paper_2601_01787_amd/build.py); "
                          "there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_size_t)
    G = ctypes.POINTER(Grid)
    L.pmsz_workspace_size.argtypes = [G, ctypes.c_int, ctypes.POINTER(sz)]
    L.pmsz_directions.argtypes = [G, vp, vp, vp]
    L.pmsz_correct.argtypes = [G, vp, vp, dbl, vp, vp, sz, i64, ctypes.POINTER(Stats), vp]
    L.pmsz_correct_mode.argtypes = [G, vp, vp, dbl, vp, ctypes.c_int, vp, sz, i64,
                                    ctypes.POINTER(Stats), vp]
    L.pmsz_batched_workspace_size.argtypes = [i32, ctypes.POINTER(Field), ctypes.POINTER(sz)]
    L.pmsz_correct_batched.argtypes = [i32, ctypes.POINTER(Field), vp, sz, i64,
                                       ctypes.POINTER(Stats), vp]
    L.pmsz_labels.argtypes = [G, vp, vp, vp, vp, sz, vp]
    L.pmsz_verify.argtypes = [G, vp, vp, vp, dbl, vp, sz, ctypes.POINTER(Report), vp]
    L.pmsz_last_timing.argtypes = [ctypes.POINTER(Timing)]
    L.pmsz_edits_workspace_size.argtypes = [G, i64, ctypes.POINTER(sz)]
    L.pmsz_edits_max_bytes.argtypes = [i64, ctypes.POINTER(sz)]
    L.pmsz_encode_edits.argtypes = [G, vp, vp, i64, vp, sz, vp, sz, ctypes.POINTER(i64),
                                    ctypes.POINTER(i64), vp]
    L.pmsz_decode_edits.argtypes = [G, vp, sz, vp, vp, sz, vp]
    L.pmsz_blocks_workspace_size.argtypes = [G, vp, ctypes.POINTER(sz)]
    L.pmsz_set_tiles_target.argtypes = [i32, i32, i32]
    L.pmsz_get_tiles_target.argtypes = [i32, i32, ctypes.POINTER(i32)]
    L.pmsz_tune_workspace_size.argtypes = [i32, ctypes.POINTER(Field), ctypes.POINTER(sz)]
    L.pmsz_tune_tiles.argtypes = [i32, ctypes.POINTER(Field), vp, i32, i32, vp, sz, vp,
                                  ctypes.POINTER(i32), vp]
    L.pmsz_correct_blocks.argtypes = [G, vp, vp, dbl, vp, i32, i64, i64, vp, sz,
                                      ctypes.POINTER(BlocksStats), vp]
    L.pmsz_last_rounds.argtypes = [ctypes.POINTER(Round), ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64)]
    L.pmsz_session_workspace_size.argtypes = [i32, ctypes.POINTER(sz)]
    L.pmsz_field_workspace_size.argtypes = [G, ctypes.POINTER(sz)]
    L.pmsz_session_create.argtypes = [i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    L.pmsz_session_add.argtypes = [vp, ctypes.POINTER(Field), i64, vp, sz,
                                   ctypes.POINTER(ctypes.c_int32)]
    L.pmsz_session_step.argtypes = [vp, i64]
    L.pmsz_session_step_ex.argtypes = [vp, i64, i32]
    L.pmsz_session_request_stop.argtypes = [vp]
    L.pmsz_session_request_stop_when_done.argtypes = [vp]
    L.pmsz_session_query.argtypes = [vp, ctypes.POINTER(i32)]
    L.pmsz_session_finished.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i32)]
    L.pmsz_session_sync.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.pmsz_session_result.argtypes = [vp, i32, ctypes.POINTER(Stats),
                                      ctypes.POINTER(ctypes.c_int32)]
    L.pmsz_session_remove.argtypes = [vp, i32]
    L.pmsz_session_destroy.argtypes = [vp]
    L.pmsz_last_labels.argtypes = [ctypes.POINTER(LabelsInfo)]
    L.pmsz_release.argtypes = []
    L.pmsz_correct_noalloc.argtypes = [G, vp, vp, dbl, vp, i64, ctypes.POINTER(Stats), vp]
    L.pmsz_probe_read.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_uint64), vp]
    L.pmsz_status_string.argtypes = [ctypes.c_int]
    L.pmsz_status_string.restype = ctypes.c_char_p
    L.pmsz_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-2]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    # the library's pinned buffers and events are freed while the HIP runtime
    # is still up (exit hooks run last-registered first, so before torch's)
    atexit.register(_release)
    return L


def _release():
    if _lib is not None:
        _lib.pmsz_release()


def _raise_if(code, allowed=(0,)):
    if code not in allowed:
        raise PmszError(code, load().pmsz_last_error().decode())


def grid_of(t):
    """pmsz_grid of a C-contiguous device tensor shaped (ny, nx) or (nz, ny, nx)."""
    if t.dtype == torch.float32:
        dt = F32
    elif t.dtype == torch.float64:
        dt = F64
    elif t.dtype == torch.uint8:
        dt = F32  # direction bytes: only the shape matters
    else:
        raise TypeError("fields must be float32 or float64, got %s" % t.dtype)
    if t.dim() == 2:
        return Grid(2, dt, t.shape[1], t.shape[0], 1)
    if t.dim() == 3:
        return Grid(3, dt, t.shape[2], t.shape[1], t.shape[0])
    raise ValueError("fields must be 2D (ny, nx) or 3D (nz, ny, nx)")


def _dev(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def workspace_size(grid, op):
    n = ctypes.c_size_t()
    _raise_if(load().pmsz_workspace_size(ctypes.byref(grid), op, ctypes.byref(n)))
    return n.value


def workspace(grid, op, device):
    """A caller-owned workspace tensor (uint8, 256-byte aligned)."""
    n = workspace_size(grid, op)
    ws = torch.empty(n + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + n]


def directions(h, out=None):
    """Direction bytes of a field: low nibble = code of n_max, high = n_min."""
    _dev(h, "field")
    grid = grid_of(h)
    if out is None:
        out = torch.empty(h.shape, dtype=torch.uint8, device=h.device)
    _dev(out, "out")
    _raise_if(load().pmsz_directions(ctypes.byref(grid), ctypes.c_void_p(h.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream(h)))
    return out


def correct(f, fhat, xi, *, inplace=False, max_iters=DEFAULT_MAX_ITERS, dirs_f=None, ws=None,
            mode="halving"):
    """Correct fhat toward f's topology within |g - f| <= xi.

    mode: "halving" (pmsz_correct) or "targeted" (pmsz_correct_mode with
    PMSZ_EDIT_TARGETED).  Returns (g, stats).  ``stats['status']`` is "OK",
    "STALLED", "NOT_CONVERGED", "NONFINITE" or "INPUT_BOUND"; argument and
    device errors raise PmszError."""
    _dev(f, "f")
    _dev(fhat, "fhat")
    if fhat.shape != f.shape or fhat.dtype != f.dtype or fhat.device != f.device:
        raise ValueError("f and fhat must match in shape, dtype and device")
    g = fhat if inplace else fhat.clone()
    grid = grid_of(f)
    emode = EDIT_MODES[mode]
    if ws is None:
        ws = workspace(grid, WS_CORRECT_TARGETED if emode else WS_CORRECT, f.device)
    st = Stats()
    dptr = ctypes.c_void_p(_dev(dirs_f, "dirs_f").data_ptr()) if dirs_f is not None else None
    code = load().pmsz_correct_mode(ctypes.byref(grid), ctypes.c_void_p(f.data_ptr()),
                                    ctypes.c_void_p(g.data_ptr()), float(xi), dptr, emode,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), int(max_iters),
                                    ctypes.byref(st), _stream(f))
    _raise_if(code, allowed=(0, 2, 3, 4, 5))
    return g, st.as_dict()


def correct_noalloc(f, fhat, xi, *, inplace=False, max_iters=DEFAULT_MAX_ITERS, dirs_f=None):
    """correct() through pmsz_correct_noalloc: the library's own static
    device scratch instead of a workspace (fields whose workspace fits
    NOALLOC_SCRATCH_BYTES).  Allocates only the output when inplace=False."""
    _dev(f, "f")
    _dev(fhat, "fhat")
    if fhat.shape != f.shape or fhat.dtype != f.dtype or fhat.device != f.device:
        raise ValueError("f and fhat must match in shape, dtype and device")
    g = fhat if inplace else fhat.clone()
    st = Stats()
    dptr = ctypes.c_void_p(_dev(dirs_f, "dirs_f").data_ptr()) if dirs_f is not None else None
    with torch.cuda.device(f.device):
        code = load().pmsz_correct_noalloc(ctypes.byref(grid_of(f)),
                                           ctypes.c_void_p(f.data_ptr()),
                                           ctypes.c_void_p(g.data_ptr()), float(xi), dptr,
                                           int(max_iters), ctypes.byref(st), _stream(f))
    _raise_if(code, allowed=(0, 2, 3, 4, 5))
    return g, st.as_dict()


def correct_batched(fields, *, max_iters=DEFAULT_MAX_ITERS):
    """Correct a list of (f, g, xi) in place (g holds fhat on entry); returns
    the list of per-field stats."""
    n = len(fields)
    arr = (Field * max(n, 1))()
    for i, (f, g, xi) in enumerate(fields):
        _dev(f, "f")
        _dev(g, "g")
        arr[i] = Field(grid_of(f), f.data_ptr(), g.data_ptr(), float(xi))
    need = ctypes.c_size_t()
    _raise_if(load().pmsz_batched_workspace_size(n, arr, ctypes.byref(need)))
    dev = fields[0][0].device if n else torch.device("cuda")
    ws = torch.empty(need.value + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    st = (Stats * max(n, 1))()
    code = load().pmsz_correct_batched(n, arr, ctypes.c_void_p(ws.data_ptr() + off),
                                       need.value, int(max_iters), st,
                                       ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    _raise_if(code, allowed=(0, 2, 3, 4, 5))
    return [st[i].as_dict() for i in range(n)]


def correct_blocks(f, fhat, xi, blocks, *, per_round=False, max_phases=1 << 20,
                   max_iters=DEFAULT_MAX_ITERS, inplace=False):
    """Decomposed-domain correction (pmsz_correct_blocks): blocks = (bx, by)
    or (bx, by, bz) virtual ranks; per_round=False runs each block to local
    convergence between exchanges, True one round.  Returns (g, stats)."""
    _dev(f, "f")
    _dev(fhat, "fhat")
    if fhat.shape != f.shape or fhat.dtype != f.dtype or fhat.device != f.device:
        raise ValueError("f and fhat must match in shape, dtype and device")
    g = fhat if inplace else fhat.clone()
    grid = grid_of(f)
    bl = (ctypes.c_int32 * 3)(*(list(blocks) + [1] * (3 - len(blocks))))
    need = ctypes.c_size_t()
    _raise_if(load().pmsz_blocks_workspace_size(ctypes.byref(grid), bl, ctypes.byref(need)))
    buf = torch.empty(need.value + 256, dtype=torch.uint8, device=f.device)
    off = (-buf.data_ptr()) % 256
    st = BlocksStats()
    code = load().pmsz_correct_blocks(ctypes.byref(grid), ctypes.c_void_p(f.data_ptr()),
                                      ctypes.c_void_p(g.data_ptr()), float(xi), bl,
                                      1 if per_round else 0, int(max_phases), int(max_iters),
                                      ctypes.c_void_p(buf.data_ptr() + off), need.value,
                                      ctypes.byref(st), _stream(f))
    _raise_if(code, allowed=(0, 2, 3, 4, 5))
    return g, st.as_dict()


TILE_TARGETS = (32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384)


def set_tiles_target(ndim, dtype, target):
    """Tiles-per-field target of the tile-height policy for (ndim, dtype)
    (torch.float32 / torch.float64); 0 restores the default rule (2048 /
    fields of a batch, between 32 and 256)."""
    _raise_if(load().pmsz_set_tiles_target(int(ndim), F32 if dtype == torch.float32 else F64,
                                           int(target)))


def get_tiles_target(ndim, dtype):
    """The set or tuned target for (ndim, dtype); 0 under the default rule."""
    t = ctypes.c_int32()
    _raise_if(load().pmsz_get_tiles_target(int(ndim), F32 if dtype == torch.float32 else F64,
                                           ctypes.byref(t)))
    return t.value


def tune_tiles(fields, candidates=TILE_TARGETS, reps=2):
    """Autotune the tile height for a batch of (f, fhat, xi) (fhat is left
    unchanged): times the correction for every candidate tiles-per-field
    target, keeps the fastest for the batch's (ndim, dtype) and returns
    (best target, {target: device ms})."""
    n = len(fields)
    arr = (Field * n)()
    for i, (f, fhat, xi) in enumerate(fields):
        _dev(f, "f")
        _dev(fhat, "fhat")
        arr[i] = Field(grid_of(f), f.data_ptr(), fhat.data_ptr(), float(xi))
    need = ctypes.c_size_t()
    _raise_if(load().pmsz_tune_workspace_size(n, arr, ctypes.byref(need)))
    dev = fields[0][0].device
    buf = torch.empty(need.value + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    cand = (ctypes.c_int32 * len(candidates))(*candidates)
    ms = (ctypes.c_double * len(candidates))()
    best = ctypes.c_int32()
    _raise_if(load().pmsz_tune_tiles(n, arr, cand, len(candidates), int(reps),
                                     ctypes.c_void_p(buf.data_ptr() + off), need.value, ms,
                                     ctypes.byref(best),
                                     ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)))
    return best.value, {int(c): ms[i] for i, c in enumerate(candidates)}


def probe_read(buf, pattern):
    """Counter-calibration probe (pmsz_probe_read): reads the bytes of the
    device tensor `buf` once as dword rows (pattern 0) or byte rows (1) and
    returns their sum as dwords / bytes."""
    _dev(buf, "buf")
    out = ctypes.c_uint64()
    _raise_if(load().pmsz_probe_read(ctypes.c_void_p(buf.data_ptr()),
                                     buf.numel() * buf.element_size(), int(pattern),
                                     ctypes.byref(out), _stream(buf)))
    return out.value


def last_timing():
    """Engine duration (HIP events on the caller's stream) and work of the last
    correction made on this thread."""
    t = Timing()
    _raise_if(load().pmsz_last_timing(ctypes.byref(t)))
    return t.as_dict()


def last_rounds():
    """Per-round records (detect and apply time, vertices examined, |F|,
    edits) of the last correction made on this thread."""
    buf = (Round * 64)()
    n = ctypes.c_int64()
    _raise_if(load().pmsz_last_rounds(buf, 64, ctypes.byref(n)))
    return [buf[i].as_dict() for i in range(min(n.value, 64))]


def field_workspace_size(grid):
    """Device bytes of one admitted field's workspace in a serving session."""
    n = ctypes.c_size_t()
    _raise_if(load().pmsz_field_workspace_size(ctypes.byref(grid), ctypes.byref(n)))
    return n.value


class Session:
    """A serving session of the C library (continuous batching): fields are
    admitted and retired between steps; each step runs the persistent
    correction kernel over every admitted, unfinished field."""

    def __init__(self, dtype, max_fields, device):
        L = load()
        self._dt = F32 if dtype == torch.float32 else F64
        n = ctypes.c_size_t()
        _raise_if(L.pmsz_session_workspace_size(int(max_fields), ctypes.byref(n)))
        buf = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self._ws = buf[off:off + n.value]
        self._stream = torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        _raise_if(L.pmsz_session_create(self._dt, int(max_fields),
                                        ctypes.c_void_p(self._ws.data_ptr()), n.value,
                                        ctypes.c_void_p(self._stream.cuda_stream),
                                        ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def add(self, f, g, xi, ws, max_iters=DEFAULT_MAX_ITERS):
        """Admit (f, g) -- g holds fhat and is corrected in place -- with its
        field workspace `ws` (a 256-byte aligned uint8 device tensor)."""
        for t, name in ((f, "f"), (g, "g"), (ws, "ws")):
            _dev(t, name)
        fld = Field(grid_of(f), f.data_ptr(), g.data_ptr(), float(xi))
        h = ctypes.c_int32()
        _raise_if(load().pmsz_session_add(self._h, ctypes.byref(fld), int(max_iters),
                                          ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          ctypes.byref(h)))
        self._keep[h.value] = (f, g, ws)
        return h.value

    def step(self, max_rounds, stop_on_done=False):
        """Launch a step (asynchronous): max_rounds rounds (< 1: until every
        field is done); stop_on_done ends it after the round in which a field
        is first seen finished."""
        _raise_if(load().pmsz_session_step_ex(self._h, int(max_rounds),
                                              STEP_STOP_ON_DONE if stop_on_done else 0))

    def request_stop(self, when_done=False):
        """Ask the step in flight to end after its current round, or (with
        when_done) after the first round that begins with one of its fields
        done."""
        if when_done:
            _raise_if(load().pmsz_session_request_stop_when_done(self._h))
        else:
            _raise_if(load().pmsz_session_request_stop(self._h))

    def running(self):
        """True while the step in flight has not ended (non-blocking)."""
        r = ctypes.c_int32()
        _raise_if(load().pmsz_session_query(self._h, ctypes.byref(r)))
        return bool(r.value)

    def finished(self):
        """[(handle, stats)] of the fields that finished in the last synced
        step."""
        n = ctypes.c_int32()
        L = load()
        _raise_if(L.pmsz_session_finished(self._h, 0, None, None, ctypes.byref(n)))
        if n.value == 0:
            return []
        hs = (ctypes.c_int32 * n.value)()
        st = (Stats * n.value)()
        _raise_if(L.pmsz_session_finished(self._h, n.value, hs, st, ctypes.byref(n)))
        return [(hs[i], st[i].as_dict()) for i in range(n.value)]

    def sync(self):
        n = ctypes.c_int32()
        _raise_if(load().pmsz_session_sync(self._h, ctypes.byref(n)))
        return n.value

    def result(self, handle):
        st = Stats()
        done = ctypes.c_int32()
        _raise_if(load().pmsz_session_result(self._h, int(handle), ctypes.byref(st),
                                             ctypes.byref(done)))
        return st.as_dict(), bool(done.value)

    def remove(self, handle):
        _raise_if(load().pmsz_session_remove(self._h, int(handle)))
        self._keep.pop(handle, None)

    def close(self):
        if self._h:
            load().pmsz_session_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone: a
        # session not closed by then is left to the process exit (the check
        # is bound at definition: module globals may be cleared by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def labels(dirs):
    """(max_label, min_label) int32 tensors: index of the extremum each vertex
    reaches along n_max / n_min."""
    _dev(dirs, "dirs")
    grid = grid_of(dirs)
    mx = torch.empty(dirs.shape, dtype=torch.int32, device=dirs.device)
    mn = torch.empty(dirs.shape, dtype=torch.int32, device=dirs.device)
    ws = workspace(grid, WS_LABELS, dirs.device)
    _raise_if(load().pmsz_labels(ctypes.byref(grid), ctypes.c_void_p(dirs.data_ptr()),
                                 ctypes.c_void_p(mx.data_ptr()), ctypes.c_void_p(mn.data_ptr()),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dirs)))
    return mx, mn


def last_labels():
    """Passes and device time of the last pmsz_labels on this thread."""
    info = LabelsInfo()
    _raise_if(load().pmsz_last_labels(ctypes.byref(info)))
    return info.as_dict()


def verify(f, g, fhat, xi):
    """Evaluation counts (Sec. V-D) of g against f."""
    _dev(f, "f")
    _dev(g, "g")
    if fhat is not None:
        _dev(fhat, "fhat")
    grid = grid_of(f)
    ws = workspace(grid, WS_VERIFY, f.device)
    rep = Report()
    _raise_if(load().pmsz_verify(ctypes.byref(grid), ctypes.c_void_p(f.data_ptr()),
                                 ctypes.c_void_p(g.data_ptr()),
                                 ctypes.c_void_p(fhat.data_ptr()) if fhat is not None else None,
                                 float(xi), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 ctypes.byref(rep), _stream(f)))
    return rep.as_dict()


def encode_edits(fhat, g, *, max_edits=None):
    """Edit stream of a corrected field g against fhat (uint8 tensor on the
    same device; format in pmsz.h).  max_edits bounds the workspace (default:
    every vertex)."""
    _dev(fhat, "fhat")
    _dev(g, "g")
    if fhat.shape != g.shape or fhat.dtype != g.dtype:
        raise ValueError("fhat and g must match")
    grid = grid_of(g)
    cap = g.numel() if max_edits is None else int(max_edits)
    need = ctypes.c_size_t()
    _raise_if(load().pmsz_edits_workspace_size(ctypes.byref(grid), cap, ctypes.byref(need)))
    ws = torch.empty(need.value + 256, dtype=torch.uint8, device=g.device)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + need.value]
    outcap = ctypes.c_size_t()
    _raise_if(load().pmsz_edits_max_bytes(cap, ctypes.byref(outcap)))
    out = torch.empty(outcap.value + 8, dtype=torch.uint8, device=g.device)
    o8 = (-out.data_ptr()) % 8
    out = out[o8:o8 + outcap.value]
    ne, nb = ctypes.c_int64(), ctypes.c_int64()
    _raise_if(load().pmsz_encode_edits(ctypes.byref(grid), ctypes.c_void_p(fhat.data_ptr()),
                                       ctypes.c_void_p(g.data_ptr()), cap,
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       ctypes.c_void_p(out.data_ptr()), out.numel(),
                                       ctypes.byref(ne), ctypes.byref(nb), _stream(g)))
    return out[:nb.value], ne.value


def decode_edits(fhat, stream):
    """The corrected field from fhat and an edit stream (device uint8 tensor)."""
    _dev(fhat, "fhat")
    _dev(stream, "stream")
    g = fhat.clone()
    grid = grid_of(g)
    s = stream
    if s.data_ptr() % 8:
        s = s.clone()
    ws = torch.empty(512, dtype=torch.uint8, device=g.device)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + 256]
    _raise_if(load().pmsz_decode_edits(ctypes.byref(grid), ctypes.c_void_p(s.data_ptr()),
                                       s.numel(), ctypes.c_void_p(g.data_ptr()),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(g)))
    return g
