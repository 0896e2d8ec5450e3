"""CPU-side checks of the C ABI: the library loads and exports every symbol
the public header declares (no kernel is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmsz.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmsz_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("pmsz_directions", "pmsz_correct", "pmsz_labels", "pmsz_verify",
                 "pmsz_correct_batched", "pmsz_workspace_size", "pmsz_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2601_01787_amd as pmsz
    lib = pmsz.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(pmsz.EXPORTS) <= set(declared_functions())


def test_host_only_calls():
    """Calls that never touch the device: status names, workspace sizes and
    argument rejection."""
    import paper_2601_01787_amd as pmsz
    lib = pmsz.load()
    assert lib.pmsz_status_string(0) == b"OK"
    assert lib.pmsz_status_string(5) == b"STALLED"
    g = pmsz.Grid(3, pmsz.F32, 512, 512, 512)
    n = pmsz.workspace_size(g, pmsz.WS_CORRECT)
    N = 512 ** 3
    # bitmap (N/8) + direction bytes (N) + target list (4 bytes for N/256 +
    # 1024 entries) + a few bytes per tile of >= 2048 vertices + fixed
    # control blocks
    lst = 4 * (N // 256 + 1024)
    assert N + N // 8 + lst <= n <= N + N // 8 + lst + 12 * (N // 2048) + 65536
    with pytest.raises(pmsz.PmszError) as e:
        pmsz.workspace_size(pmsz.Grid(2, pmsz.F32, 4, 4, 3), pmsz.WS_CORRECT)
    assert e.value.status == 1
    with pytest.raises(pmsz.PmszError):
        pmsz.workspace_size(pmsz.Grid(3, pmsz.F32, 1 << 11, 1 << 11, 1 << 10), pmsz.WS_CORRECT)
    with pytest.raises(pmsz.PmszError):
        pmsz.workspace_size(pmsz.Grid(3, 7, 4, 4, 4), pmsz.WS_CORRECT)
    st = pmsz.Stats()
    # NULL pointers are rejected before any device work
    code = lib.pmsz_correct(ctypes.byref(g), None, None, 0.1, None, None, 0, 10,
                            ctypes.byref(st), None)
    assert code == 1
    assert b"NULL" in lib.pmsz_last_error()
    code = lib.pmsz_correct_noalloc(ctypes.byref(g), None, None, 0.1, None, 10,
                                    ctypes.byref(st), None)
    assert code == 1
    # a field whose workspace exceeds the static scratch is refused before any
    # device call (the pointers are never touched)
    fake = ctypes.c_void_p(256)
    code = lib.pmsz_correct_noalloc(ctypes.byref(g), fake, fake, 0.1, None, 10,
                                    ctypes.byref(st), None)
    assert code == 6 and b"allocation-free correction" in lib.pmsz_last_error()


def test_blocks_workspace_size_host_only():
    """pmsz_blocks_workspace_size: per block copies of f and g (value size),
    direction bytes, plus the engine workspace of the block fields; bad block
    counts are rejected."""
    import paper_2601_01787_amd as pmsz
    lib = pmsz.load()
    g = pmsz.Grid(3, pmsz.F32, 64, 64, 64)
    b = (ctypes.c_int32 * 3)(2, 2, 2)
    n = ctypes.c_size_t()
    assert lib.pmsz_blocks_workspace_size(ctypes.byref(g), b, ctypes.byref(n)) == 0
    copies = 8 * 33 ** 3
    assert n.value >= copies * (4 + 4 + 1)
    assert n.value <= copies * (4 + 4 + 1) * 2 + (1 << 22)
    for bad in ((65, 1, 1), (0, 1, 1), (1, 1, 2)):
        gg = pmsz.Grid(3, pmsz.F32, 64, 64, 64) if bad[2] < 2 else pmsz.Grid(2, pmsz.F32, 64, 64, 1)
        assert lib.pmsz_blocks_workspace_size(ctypes.byref(gg), (ctypes.c_int32 * 3)(*bad),
                                              ctypes.byref(n)) == 1


def test_tiles_target_host_only():
    """The tile-height policy: per (ndim, dtype), 0 restores the default rule
    (reported as 0), bad arguments are rejected, and workspace sizes do not
    depend on it."""
    import paper_2601_01787_amd as pmsz
    lib = pmsz.load()
    t = ctypes.c_int32()
    assert lib.pmsz_get_tiles_target(3, pmsz.F32, ctypes.byref(t)) == 0 and t.value == 0
    g = pmsz.Grid(3, pmsz.F32, 300, 200, 100)
    before = pmsz.workspace_size(g, pmsz.WS_CORRECT)
    assert lib.pmsz_set_tiles_target(3, pmsz.F32, 64) == 0
    assert lib.pmsz_get_tiles_target(3, pmsz.F32, ctypes.byref(t)) == 0 and t.value == 64
    assert lib.pmsz_get_tiles_target(2, pmsz.F32, ctypes.byref(t)) == 0 and t.value == 0
    assert pmsz.workspace_size(g, pmsz.WS_CORRECT) == before
    assert lib.pmsz_set_tiles_target(3, pmsz.F32, 0) == 0
    assert lib.pmsz_get_tiles_target(3, pmsz.F32, ctypes.byref(t)) == 0 and t.value == 0
    assert lib.pmsz_set_tiles_target(4, pmsz.F32, 64) == 1
    assert lib.pmsz_set_tiles_target(3, 9, 64) == 1
    assert lib.pmsz_set_tiles_target(3, pmsz.F32, -1) == 1


def test_tune_cache_is_read_before_the_first_target(tmp_path):
    """PMSZ_TUNE_CACHE names a JSON file of tuned tiles-per-field targets: its
    entries are the process's targets until set otherwise, absent keys keep
    the default, and a malformed file is ignored (host-only calls)."""
    import json
    import subprocess
    import sys
    code = ("import paper_2601_01787_amd as p, torch; "
            "print(p.get_tiles_target(3, torch.float32), p.get_tiles_target(2, torch.float64), "
            "p.get_tiles_target(2, torch.float32), p.get_tiles_target(3, torch.float64))")

    def targets(text):
        cache = tmp_path / "tune.json"
        cache.write_text(text)
        env = dict(os.environ, PMSZ_TUNE_CACHE=str(cache))
        out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, check=True,
                             capture_output=True, text=True).stdout
        return [int(v) for v in out.split()]

    assert targets(json.dumps({"3d_f32": 96, "2d_f64": 7})) == [96, 7, 0, 0]
    assert targets('{"2d_f32" :  40 ,\n "3d_f64": 0}') == [0, 0, 40, 0]
    assert targets("not json at all") == [0, 0, 0, 0]
