"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rxphy.h")
LIB = os.environ.get("RXPHY_LIBRARY") or os.path.join(ROOT, "paper_2603_20481_amd", "librxphy.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rxphy_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librxphy.so not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_stage_calls():
    names = declared_functions()
    for n in ("rxphy_fft", "rxphy_csi", "rxphy_detect", "rxphy_demod", "rxphy_backward",
              "rxphy_workspace_bytes", "rxphy_status_string", "rxphy_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


class Frame(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("K", ctypes.c_int32), ("n_fft", ctypes.c_int32),
                ("n_sc", ctypes.c_int32), ("n_sym", ctypes.c_int32), ("cp_len", ctypes.c_int32),
                ("qam_bits", ctypes.c_int32), ("detector", ctypes.c_int32), ("n0", ctypes.c_float)]


GOOD = dict(M=64, K=16, n_fft=2048, n_sc=1200, n_sym=14, cp_len=0, qam_bits=4, detector=0, n0=1.0)


def frame(**kw):
    d = dict(GOOD)
    d.update(kw)
    return Frame(**d)


BAD = [
    (dict(K=0), 1), (dict(K=17), 2), (dict(M=65), 2), (dict(K=9, M=8), 1),
    (dict(n_fft=1000), 1), (dict(n_fft=256), 2), (dict(n_fft=8192), 2),
    (dict(n_sc=15), 1), (dict(n_sc=2049), 1), (dict(n_sym=1), 1), (dict(n_sym=18), 2),
    (dict(cp_len=-1), 1), (dict(cp_len=2049), 1), (dict(qam_bits=3), 1), (dict(detector=2), 1),
    (dict(n0=0.0), 1), (dict(n0=float("nan")), 1), (dict(n0=float("inf")), 1),
]


@pytest.mark.parametrize("kw,code", BAD)
def test_bad_shapes_rejected_before_launch(lib, kw, code):
    fr = frame(**kw)
    p = ctypes.c_void_p(16)      # never dereferenced: validation fails first
    lib.rxphy_fft.restype = ctypes.c_int
    assert lib.rxphy_fft(ctypes.byref(fr), 1, p, p, None) == code
    lib.rxphy_last_error.restype = ctypes.c_char_p
    assert lib.rxphy_last_error()  # a message was recorded
    lib.rxphy_demod.restype = ctypes.c_int
    assert lib.rxphy_demod(ctypes.byref(fr), 1, p, p, p, None) == code


def test_null_pointers_and_counts(lib):
    fr = frame()
    p = ctypes.c_void_p(16)
    assert lib.rxphy_fft(None, 1, p, p, None) == 1
    assert lib.rxphy_fft(ctypes.byref(fr), -1, p, p, None) == 1
    assert lib.rxphy_fft(ctypes.byref(fr), 1, None, p, None) == 1
    assert lib.rxphy_csi(ctypes.byref(fr), 1, p, None, p, None) == 1
    # zero frames is a valid no-op that touches nothing
    assert lib.rxphy_fft(ctypes.byref(fr), 0, None, None, None) == 0
    assert lib.rxphy_demod(ctypes.byref(fr), 0, None, None, None, None) == 0


def test_detect_argument_checks(lib):
    fr = frame()
    p = ctypes.c_void_p(16)
    lib.rxphy_detect.argtypes = [ctypes.POINTER(Frame), ctypes.c_int32] + [ctypes.c_void_p] * 5 + \
        [ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.rxphy_detect.restype = ctypes.c_int
    assert lib.rxphy_detect(ctypes.byref(fr), 1, p, p, p, p, p, 7, 1e3, None, 0, None) == 1
    assert lib.rxphy_detect(ctypes.byref(fr), 1, p, p, p, p, p, 1, -1.0, None, 0, None) == 1
    assert lib.rxphy_detect(ctypes.byref(fr), 1, None, p, p, p, p, 0, 1e3, None, 0, None) == 1
    assert lib.rxphy_detect(ctypes.byref(fr), 0, None, None, None, None, None, 0, 1e3, None, 0, None) == 0


def test_fused_call_checks(lib):
    """rxphy_csi_detect_demod: argument, workspace, alignment and frame-count
    errors come back before any HIP call (the pointers here are never
    dereferenced)."""
    fr = frame(M=64, K=16, n_fft=2048, n_sc=1200, n_sym=14, qam_bits=4)
    p = ctypes.c_void_p(256)
    f = lib.rxphy_csi_detect_demod
    f.argtypes = [ctypes.POINTER(Frame), ctypes.c_int32] + [ctypes.c_void_p] * 6 + \
        [ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    f.restype = ctypes.c_int
    lib.rxphy_workspace_bytes.argtypes = [ctypes.POINTER(Frame), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.rxphy_workspace_bytes.restype = ctypes.c_size_t
    need = lib.rxphy_workspace_bytes(ctypes.byref(fr), 1, 3, 0)
    assert need == 75 * 2304                         # one factor record per 16-subcarrier tile
    big = 1 << 40
    assert f(ctypes.byref(fr), 1, p, p, None, p, p, p, 0, 1e3, p, need - 1, None) == 3      # workspace
    assert f(ctypes.byref(fr), 1, p, p, None, p, p, None, 0, 1e3, p, need, None) == 1       # llr NULL
    assert f(ctypes.byref(fr), 1, p, p, None, p, p, p, 9, 1e3, p, need, None) == 1          # precision
    assert f(ctypes.byref(fr), 1, p, p, None, p, p, p, 0, 1e3, ctypes.c_void_p(260), need, None) == 3
    assert f(ctypes.byref(fr), 70000, p, p, None, p, p, p, 0, 1e3, p, big, None) == 2       # grid limit
    assert f(ctypes.byref(fr), 0, None, None, None, None, None, None, 0, 1e3, None, 0, None) == 0


def test_noalloc_call_rejects_work_beyond_its_scratch(lib):
    """rxphy_csi_detect_demod_noalloc: a call whose workspace would exceed the
    library's 32 MiB scratch fails with RXPHY_EWORKSPACE before any HIP call;
    194 frames of 64 x 16 with 1200 subcarriers is the most that fits."""
    fr = frame(M=64, K=16, n_fft=2048, n_sc=1200, n_sym=14, qam_bits=4)
    p = ctypes.c_void_p(256)
    f = lib.rxphy_csi_detect_demod_noalloc
    f.argtypes = [ctypes.POINTER(Frame), ctypes.c_int32] + [ctypes.c_void_p] * 6 + \
        [ctypes.c_int32, ctypes.c_float, ctypes.c_void_p]
    f.restype = ctypes.c_int
    lib.rxphy_workspace_bytes.argtypes = [ctypes.POINTER(Frame), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.rxphy_workspace_bytes.restype = ctypes.c_size_t
    cap = 32 << 20
    assert lib.rxphy_workspace_bytes(ctypes.byref(fr), 194, 3, 0) <= cap
    assert lib.rxphy_workspace_bytes(ctypes.byref(fr), 195, 3, 0) > cap
    assert f(ctypes.byref(fr), 195, p, p, None, p, p, p, 0, 1e3, None) == 3
    lib.rxphy_last_error.restype = ctypes.c_char_p
    assert b"scratch" in lib.rxphy_last_error()
    assert f(ctypes.byref(fr), 1, p, p, None, p, p, p, 9, 1e3, None) == 1          # precision
    assert f(ctypes.byref(frame(K=17)), 1, p, p, None, p, p, p, 0, 1e3, None) == 2
    assert f(ctypes.byref(fr), 0, None, None, None, None, None, None, 0, 1e3, None) == 0


def test_ldpc_code_checks(lib):
    """rxphy_ldpc_code_create rejects bad base matrices before any HIP call;
    rxphy_ldpc_decode rejects bad arguments before any launch."""
    import numpy as np
    f = lib.rxphy_ldpc_code_create
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
    f.restype = ctypes.c_int
    h = ctypes.c_void_p()

    def create(b, z):
        b = np.ascontiguousarray(np.asarray(b, dtype=np.int16))
        return f(b.ctypes.data, b.shape[0], b.shape[1], z, ctypes.byref(h))
    ok = np.array([[0, 1, 0, -1], [2, -1, 0, 0]])
    assert create(ok, 0) == 1                                   # z < 1
    assert create(ok, 385) == 2                                 # z > 384
    assert create(np.array([[0, 5, 0, -1], [2, -1, 0, 0]]), 4) == 1    # shift >= z
    assert create(np.array([[0, -2, 0, -1], [2, -1, 0, 0]]), 4) == 1   # entry < -1
    assert create(np.array([[0, -1, -1, -1], [2, -1, 0, 0]]), 4) == 1  # a degree-1 row
    assert create(np.zeros((2, 28), np.int16), 4) == 2          # degree 28 > 27
    assert create(np.zeros((3, 3), np.int16), 4) == 1           # mb >= nb
    assert create(np.zeros((2, 101), np.int16) - 1 + np.eye(2, 101, dtype=np.int16) * 1 +
                  np.eye(2, 101, 1, dtype=np.int16), 384) == 2  # N = 38784 > 38400
    assert f(None, 2, 4, 4, ctypes.byref(h)) == 1
    d = lib.rxphy_ldpc_decode
    d.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_float] + \
        [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_void_p]
    d.restype = ctypes.c_int
    p = ctypes.c_void_p(256)
    assert d(None, 1, p, 5, 0.75, p, p, p, p, 1 << 20, None) == 1
    lib.rxphy_ldpc_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.rxphy_ldpc_workspace_bytes.restype = ctypes.c_size_t
    assert lib.rxphy_ldpc_workspace_bytes(None, 4) == 0


def test_status_strings(lib):
    lib.rxphy_status_string.restype = ctypes.c_char_p
    assert lib.rxphy_status_string(0) == b"RXPHY_OK"
    assert lib.rxphy_status_string(3) == b"RXPHY_EWORKSPACE"


def test_python_binding_refuses_without_library(tmp_path):
    import paper_2603_20481_amd as rx
    with pytest.raises(rx.RxphyError):
        rx._lib = None
        rx.load(str(tmp_path / "missing.so"))
    rx._lib = None


class Tiles(ctypes.Structure):
    _fields_ = [("fft_iters", ctypes.c_int32), ("csi_tiles", ctypes.c_int32),
                ("det_tiles", ctypes.c_int32), ("det_kp", ctypes.c_int32),
                ("dem_groups", ctypes.c_int32)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("grid", ctypes.c_int32), ("spin_limit", ctypes.c_uint32),
                ("fuse_csi", ctypes.c_int32), ("fuse_demod", ctypes.c_int32)]


def _plan_create(lib, frames, tiles=None, opts=None):
    lib.rxphy_plan_create.restype = ctypes.c_int
    arr = (Frame * len(frames))(*frames) if frames else None
    tarr = (Tiles * len(tiles))(*tiles) if tiles else None
    h = ctypes.c_void_p(123)
    st = lib.rxphy_plan_create(arr, len(frames), tarr, ctypes.byref(opts) if opts else None,
                               ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("case,code", [
    ("no frames", 1), ("bad frame", 1), ("unsupported frame", 2), ("negative tile", 1),
    ("kp below K", 1), ("kp not a size", 1), ("bad stage mask", 1), ("negative grid", 1),
    ("bad fuse_csi", 1), ("bad fuse_demod", 1),
])
def test_plan_create_rejects_before_touching_the_device(lib, case, code):
    fr = [frame(), frame(M=8, K=2, n_fft=512, n_sc=300, qam_bits=2)]
    tiles, opts = None, None
    if case == "no frames":
        fr = []
    elif case == "bad frame":
        fr[1] = frame(qam_bits=5)
    elif case == "unsupported frame":
        fr[0] = frame(K=17)
    elif case == "negative tile":
        tiles = [Tiles(0, 0, -1, 0, 0), Tiles()]
    elif case == "kp below K":
        tiles = [Tiles(0, 0, 0, 8, 0), Tiles()]          # frame 0 has K = 16
    elif case == "kp not a size":
        tiles = [Tiles(), Tiles(0, 0, 0, 5, 0)]
    elif case == "bad stage mask":
        opts = PlanOptions(16, 0, 0)
    elif case == "negative grid":
        opts = PlanOptions(0, -1, 0)
    elif case == "bad fuse_csi":
        opts = PlanOptions(0, 0, 0, 2, 0)
    elif case == "bad fuse_demod":
        opts = PlanOptions(0, 0, 0, 0, 2)
    st, h = _plan_create(lib, fr, tiles, opts)
    assert st == code, (case, st)
    assert h.value is None                              # *plan cleared on failure
    lib.rxphy_last_error.restype = ctypes.c_char_p
    assert lib.rxphy_last_error()
