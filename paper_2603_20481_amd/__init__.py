"""Python face of librxphy, the MI355X OFDM massive-MIMO uplink receiver.

Argument marshalling only: every stage runs in the HIP kernels of
``librxphy.so`` (built in-tree by ``__graft_entry__.build()``), launched on
torch's current stream.  PyTorch provides device memory and streams.  There
is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# RXPHY_LIBRARY selects another build of the library (e.g. the host-sanitized one)
LIB_PATH = os.environ.get("RXPHY_LIBRARY") or os.path.join(_HERE, "librxphy.so")

ZF, MMSE = 0, 1
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
FLAG_REFINED, FLAG_BREAKDOWN, FLAG_NONFINITE = 1, 2, 4
WS_DETECT, WS_BACKWARD, WS_CSI_DETECT, WS_CSI_DETECT_DEMOD, WS_PRECODE = 0, 1, 2, 3, 4


class RxphyError(RuntimeError):
    pass


class _Frame(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("K", ctypes.c_int32), ("n_fft", ctypes.c_int32),
                ("n_sc", ctypes.c_int32), ("n_sym", ctypes.c_int32), ("cp_len", ctypes.c_int32),
                ("qam_bits", ctypes.c_int32), ("detector", ctypes.c_int32), ("n0", ctypes.c_float)]


class _Saved(ctypes.Structure):
    _fields_ = [("yf", ctypes.c_void_p), ("h", ctypes.c_void_p), ("xt", ctypes.c_void_p), ("nu", ctypes.c_void_p)]


class _Tiles(ctypes.Structure):
    _fields_ = [("fft_iters", ctypes.c_int32), ("csi_tiles", ctypes.c_int32),
                ("det_tiles", ctypes.c_int32), ("det_kp", ctypes.c_int32),
                ("dem_groups", ctypes.c_int32)]


class _PlanOptions(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("grid", ctypes.c_int32), ("spin_limit", ctypes.c_uint32),
                ("fuse_csi", ctypes.c_int32), ("fuse_demod", ctypes.c_int32)]


_TENSORS = ("x", "pilots", "yf", "h", "xt", "nu", "flags", "llr")


class _Offsets(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in _TENSORS]


class _Batch(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in _TENSORS]


@dataclasses.dataclass(frozen=True)
class Frame:
    """Shape of one frame (mirrors ``rxphy_frame``)."""
    M: int
    K: int
    n_fft: int
    n_sc: int
    n_sym: int = 14
    cp_len: int = 0
    qam_bits: int = 2
    detector: int = ZF
    n0: float = 1.0

    @property
    def n_data(self) -> int:
        return self.n_sym - 1

    def c(self) -> _Frame:
        return _Frame(self.M, self.K, self.n_fft, self.n_sc, self.n_sym, self.cp_len,
                      self.qam_bits, self.detector, self.n0)

    @staticmethod
    def of(shape, detector=ZF, n0=1.0) -> "Frame":
        """From any object with M, K, n_fft, n_sc, n_sym, cp_len, qam_bits."""
        return Frame(shape.M, shape.K, shape.n_fft, shape.n_sc, shape.n_sym, shape.cp_len,
                     shape.qam_bits, int(detector), float(n0))


class _SenseConfig(ctypes.Structure):
    _fields_ = [("n_fft", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("sg_window", ctypes.c_int32),
                ("sg_order", ctypes.c_int32), ("psd_factor", ctypes.c_float), ("bins", ctypes.c_int32)]


_SENSE_OUT = ("tf", "psd", "psd_smooth", "floor", "otsu_bin", "mask", "mask_mo")


class _SenseOutputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in _SENSE_OUT]


class _Metrics(ctypes.Structure):
    _fields_ = [("n_t", ctypes.c_int32), ("n_f", ctypes.c_int32), ("p_d", ctypes.c_double),
                ("p_fa", ctypes.c_double), ("mean_iou", ctypes.c_double)]


class _StreamHost(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("pilots", ctypes.c_void_p), ("llr", ctypes.c_void_p),
                ("nu", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class _LatencySummary(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("on_time", ctypes.c_int64), ("meets_99", ctypes.c_int32),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("mean_us", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librxphy.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RxphyError("librxphy.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I32, F32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
    FR = ctypes.POINTER(_Frame)
    sigs = {
        "rxphy_fft": [FR, I32, P, P, P],
        "rxphy_fft_sc16": [FR, I32, P, F32, P, P],
        "rxphy_csi": [FR, I32, P, P, P, P],
        "rxphy_detect": [FR, I32, P, P, P, P, P, I32, F32, P, SZ, P],
        "rxphy_csi_detect": [FR, I32, P, P, P, P, P, I32, F32, P, SZ, P],
        "rxphy_csi_detect_demod": [FR, I32, P, P, P, P, P, P, I32, F32, P, SZ, P],
        "rxphy_csi_detect_demod_noalloc": [FR, I32, P, P, P, P, P, P, I32, F32, P],
        "rxphy_modulate": [FR, I32, P, P, P],
        "rxphy_precode": [FR, I32, P, P, P, P, P, P, SZ, ctypes.c_uint32, P],
        "rxphy_modulate_precode": [FR, I32, P, P, P, P, P, P, SZ, ctypes.c_uint32, P],
        "rxphy_ifft": [FR, ctypes.c_int64, P, P, P],
        "rxphy_ifft_sc16": [FR, ctypes.c_int64, P, F32, P, P],
        "rxphy_demod": [FR, I32, P, P, P, P],
        "rxphy_backward": [FR, I32, P, P, ctypes.POINTER(_Saved), P, P, P, P, SZ, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    PL = ctypes.c_void_p
    plan_sigs = {
        "rxphy_plan_create": [FR, I32, ctypes.POINTER(_Tiles), ctypes.POINTER(_PlanOptions),
                              ctypes.POINTER(PL)],
        "rxphy_plan_layout": [PL, ctypes.POINTER(_Offsets), ctypes.POINTER(_Offsets)],
        "rxphy_plan_info": [PL, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(I32)],
        "rxphy_plan_forward": [PL, ctypes.POINTER(_Batch), P],
        "rxphy_plan_graph": [PL, ctypes.POINTER(_Batch)],
        "rxphy_plan_replay": [PL, P],
        "rxphy_plan_device_status": [PL, ctypes.POINTER(ctypes.c_uint32)],
    }
    for name, args in plan_sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    ST = ctypes.c_void_p
    stream_sigs = {
        "rxphy_stream_create": [FR, I32, I32, I32, F32, ctypes.POINTER(ST)],
        "rxphy_stream_host_buffers": [ST, I32, ctypes.POINTER(_StreamHost)],
        "rxphy_stream_acquire": [ST, ctypes.POINTER(I32)],
        "rxphy_stream_submit": [ST, I32, ctypes.c_int64, P, P, P, P, P],
        "rxphy_stream_drain": [ST],
        "rxphy_stream_latencies": [ST, ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64)],
        "rxphy_stream_reset_latencies": [ST],
        "rxphy_latency_summarize": [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_double,
                                    ctypes.POINTER(_LatencySummary)],
    }
    for name, args in stream_sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    SC = ctypes.POINTER(_SenseConfig)
    lib.rxphy_sense_workspace_bytes.argtypes = [SC, I32]
    lib.rxphy_sense_workspace_bytes.restype = SZ
    lib.rxphy_sense.argtypes = [SC, I32, P, ctypes.POINTER(_SenseOutputs), P, P, I32, P, SZ, P]
    lib.rxphy_sense.restype = ctypes.c_int
    lib.rxphy_box_metrics.argtypes = [P, I32, P, I32, ctypes.c_double, P, ctypes.POINTER(_Metrics)]
    lib.rxphy_box_metrics.restype = ctypes.c_int
    lib.rxphy_savgol_weights.argtypes = [I32, I32, P]
    lib.rxphy_savgol_weights.restype = ctypes.c_int
    lib.rxphy_stream_destroy.argtypes = [ST]
    lib.rxphy_stream_destroy.restype = None
    lib.rxphy_clock_ns.argtypes = []
    lib.rxphy_clock_ns.restype = ctypes.c_int64
    lib.rxphy_plan_destroy.argtypes = [PL]
    lib.rxphy_plan_destroy.restype = None
    LC = ctypes.c_void_p
    lib.rxphy_ldpc_code_create.argtypes = [P, I32, I32, I32, ctypes.POINTER(LC)]
    lib.rxphy_ldpc_code_create.restype = ctypes.c_int
    lib.rxphy_ldpc_code_destroy.argtypes = [LC]
    lib.rxphy_ldpc_code_destroy.restype = None
    lib.rxphy_ldpc_workspace_bytes.argtypes = [LC, I32]
    lib.rxphy_ldpc_workspace_bytes.restype = SZ
    lib.rxphy_ldpc_decode.argtypes = [LC, I32, P, I32, F32, P, P, P, P, SZ, P]
    lib.rxphy_ldpc_decode.restype = ctypes.c_int
    lib.rxphy_workspace_bytes.argtypes = [FR, I32, I32, I32]
    lib.rxphy_workspace_bytes.restype = SZ
    lib.rxphy_status_string.argtypes = [ctypes.c_int]
    lib.rxphy_status_string.restype = ctypes.c_char_p
    lib.rxphy_last_error.argtypes = []
    lib.rxphy_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st: int, what: str):
    if st != 0:
        lib = load()
        raise RxphyError("%s: %s (%s)" % (what, lib.rxphy_status_string(st).decode(),
                                          lib.rxphy_last_error().decode()))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, shape, dtype):
    if t.device.type != "cuda":
        raise RxphyError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise RxphyError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise RxphyError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise RxphyError("%s must be contiguous" % name)


def _nf(t):
    return t.shape[0]


def _empty(shape, dtype, like):
    return torch.empty(shape, dtype=dtype, device=like.device)


# ------------------------------------------------------------------- stages
def fft(fr: Frame, x, yf=None):
    """x c64 [F][M][n_sym][cp+N] -> yf c64 [F][M][n_sym][n_sc]."""
    F = _nf(x)
    _need(x, "x", (F, fr.M, fr.n_sym, fr.cp_len + fr.n_fft), torch.complex64)
    if yf is None:
        yf = _empty((F, fr.M, fr.n_sym, fr.n_sc), torch.complex64, x)
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _check(load().rxphy_fft(ctypes.byref(fr.c()), F, _ptr(x), _ptr(yf), _stream()), "rxphy_fft")
    return yf



def fft_sc16(fr: Frame, x, scale: float, yf=None):
    """x i16 [F][M][n_sym][cp+N][2] (I, Q) with value = integer * scale ->
    yf c64 [F][M][n_sym][n_sc]."""
    F = _nf(x)
    _need(x, "x", (F, fr.M, fr.n_sym, fr.cp_len + fr.n_fft, 2), torch.int16)
    if yf is None:
        yf = _empty((F, fr.M, fr.n_sym, fr.n_sc), torch.complex64, x)
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _check(load().rxphy_fft_sc16(ctypes.byref(fr.c()), F, _ptr(x), float(scale), _ptr(yf), _stream()),
           "rxphy_fft_sc16")
    return yf


def csi(fr: Frame, yf, pilots, h=None):
    """yf c64 [F][M][n_sym][n_sc], pilots c64 [F][n_sc] -> h c64 [F][M][K][n_sc]."""
    F = _nf(yf)
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _need(pilots, "pilots", (F, fr.n_sc), torch.complex64)
    if h is None:
        h = _empty((F, fr.M, fr.K, fr.n_sc), torch.complex64, yf)
    _need(h, "h", (F, fr.M, fr.K, fr.n_sc), torch.complex64)
    _check(load().rxphy_csi(ctypes.byref(fr.c()), F, _ptr(yf), _ptr(pilots), _ptr(h), _stream()),
           "rxphy_csi")
    return h


def workspace_bytes(fr: Frame, n_frames: int, which: int, precision: str = "fp32") -> int:
    return int(load().rxphy_workspace_bytes(ctypes.byref(fr.c()), n_frames, which,
                                            PRECISIONS[precision]))


def detect(fr: Frame, h, yf, precision: str = "fp32", cond_threshold: float = 1e3,
           xt=None, nu=None, flags=None, ws=None):
    """-> (xt c64 [F][K][D][n_sc], nu f32 [F][K][n_sc], flags u8 [F][n_sc])."""
    F = _nf(h)
    D = fr.n_data
    _need(h, "h", (F, fr.M, fr.K, fr.n_sc), torch.complex64)
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    xt = _empty((F, fr.K, D, fr.n_sc), torch.complex64, h) if xt is None else xt
    nu = _empty((F, fr.K, fr.n_sc), torch.float32, h) if nu is None else nu
    flags = _empty((F, fr.n_sc), torch.uint8, h) if flags is None else flags
    _need(xt, "xt", (F, fr.K, D, fr.n_sc), torch.complex64)
    _need(nu, "nu", (F, fr.K, fr.n_sc), torch.float32)
    _need(flags, "flags", (F, fr.n_sc), torch.uint8)
    need = workspace_bytes(fr, F, WS_DETECT, precision)
    if need and ws is None:
        ws = _empty((need,), torch.uint8, h)
    _check(load().rxphy_detect(ctypes.byref(fr.c()), F, _ptr(h), _ptr(yf), _ptr(xt), _ptr(nu),
                               _ptr(flags), PRECISIONS[precision], float(cond_threshold),
                               _ptr(ws), ws.numel() if ws is not None else 0, _stream()),
           "rxphy_detect")
    return xt, nu, flags


def csi_detect(fr: Frame, yf, pilots, precision: str = "fp32", cond_threshold: float = 1e3,
               xt=None, nu=None, flags=None, ws=None):
    """csi and detect fused (H never stored); same outputs as detect(fr, csi(fr, yf, pilots), yf)."""
    F = _nf(yf)
    D = fr.n_data
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _need(pilots, "pilots", (F, fr.n_sc), torch.complex64)
    xt = _empty((F, fr.K, D, fr.n_sc), torch.complex64, yf) if xt is None else xt
    nu = _empty((F, fr.K, fr.n_sc), torch.float32, yf) if nu is None else nu
    flags = _empty((F, fr.n_sc), torch.uint8, yf) if flags is None else flags
    _need(xt, "xt", (F, fr.K, D, fr.n_sc), torch.complex64)
    _need(nu, "nu", (F, fr.K, fr.n_sc), torch.float32)
    _need(flags, "flags", (F, fr.n_sc), torch.uint8)
    need = workspace_bytes(fr, F, WS_CSI_DETECT, precision)
    if need and ws is None:
        ws = _empty((need,), torch.uint8, yf)
    _check(load().rxphy_csi_detect(ctypes.byref(fr.c()), F, _ptr(yf), _ptr(pilots), _ptr(xt), _ptr(nu),
                                   _ptr(flags), PRECISIONS[precision], float(cond_threshold),
                                   _ptr(ws), ws.numel() if ws is not None else 0, _stream()),
           "rxphy_csi_detect")
    return xt, nu, flags


def csi_detect_demod(fr: Frame, yf, pilots, precision: str = "fp32", cond_threshold: float = 1e3,
                     want_xt: bool = False, llr=None, nu=None, flags=None, xt=None, ws=None):
    """csi, detect and demod fused -> (llr, nu, flags, xt or None); the same
    llr, nu and flags as demod(fr, *csi_detect(fr, yf, pilots)[:2])."""
    F = _nf(yf)
    D = fr.n_data
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _need(pilots, "pilots", (F, fr.n_sc), torch.complex64)
    llr = _empty((F, fr.K, D, fr.n_sc, fr.qam_bits), torch.float32, yf) if llr is None else llr
    nu = _empty((F, fr.K, fr.n_sc), torch.float32, yf) if nu is None else nu
    flags = _empty((F, fr.n_sc), torch.uint8, yf) if flags is None else flags
    if xt is None and want_xt:
        xt = _empty((F, fr.K, D, fr.n_sc), torch.complex64, yf)
    _need(llr, "llr", (F, fr.K, D, fr.n_sc, fr.qam_bits), torch.float32)
    _need(nu, "nu", (F, fr.K, fr.n_sc), torch.float32)
    _need(flags, "flags", (F, fr.n_sc), torch.uint8)
    if xt is not None:
        _need(xt, "xt", (F, fr.K, D, fr.n_sc), torch.complex64)
    need = workspace_bytes(fr, F, WS_CSI_DETECT_DEMOD, precision)
    if need and ws is None:
        ws = _empty((need,), torch.uint8, yf)
    _check(load().rxphy_csi_detect_demod(ctypes.byref(fr.c()), F, _ptr(yf), _ptr(pilots),
                                         _ptr(xt) if xt is not None else None, _ptr(nu), _ptr(flags),
                                         _ptr(llr), PRECISIONS[precision], float(cond_threshold),
                                         _ptr(ws), ws.numel() if ws is not None else 0, _stream()),
           "rxphy_csi_detect_demod")
    return llr, nu, flags, xt


def csi_detect_demod_noalloc(fr: Frame, yf, pilots, precision: str = "fp32", cond_threshold: float = 1e3,
                             llr=None, nu=None, flags=None, xt=None):
    """csi_detect_demod with the library's own per-GPU scratch as workspace
    (the call allocates nothing itself; outputs are allocated here only when
    not passed in) -> (llr, nu, flags, xt or None)."""
    F = _nf(yf)
    D = fr.n_data
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _need(pilots, "pilots", (F, fr.n_sc), torch.complex64)
    llr = _empty((F, fr.K, D, fr.n_sc, fr.qam_bits), torch.float32, yf) if llr is None else llr
    nu = _empty((F, fr.K, fr.n_sc), torch.float32, yf) if nu is None else nu
    flags = _empty((F, fr.n_sc), torch.uint8, yf) if flags is None else flags
    _need(llr, "llr", (F, fr.K, D, fr.n_sc, fr.qam_bits), torch.float32)
    _need(nu, "nu", (F, fr.K, fr.n_sc), torch.float32)
    _need(flags, "flags", (F, fr.n_sc), torch.uint8)
    if xt is not None:
        _need(xt, "xt", (F, fr.K, D, fr.n_sc), torch.complex64)
    _check(load().rxphy_csi_detect_demod_noalloc(ctypes.byref(fr.c()), F, _ptr(yf), _ptr(pilots),
                                                 _ptr(xt) if xt is not None else None, _ptr(nu), _ptr(flags),
                                                 _ptr(llr), PRECISIONS[precision], float(cond_threshold),
                                                 _stream()),
           "rxphy_csi_detect_demod_noalloc")
    return llr, nu, flags, xt


# ------------------------------------------------------------------ downlink
def modulate(fr: Frame, bits, sym=None):
    """bits u8 [F][K][D][n_sc][qam_bits] (0/1, b0 first) -> QAM points c64 [F][K][D][n_sc]."""
    F = _nf(bits)
    D = fr.n_data
    _need(bits, "bits", (F, fr.K, D, fr.n_sc, fr.qam_bits), torch.uint8)
    sym = _empty((F, fr.K, D, fr.n_sc), torch.complex64, bits) if sym is None else sym
    _need(sym, "sym", (F, fr.K, D, fr.n_sc), torch.complex64)
    _check(load().rxphy_modulate(ctypes.byref(fr.c()), F, _ptr(bits), _ptr(sym), _stream()), "rxphy_modulate")
    return sym


PRECODE_REUSE_FACTORS = 1


def precode(fr: Frame, yf, pilots, sym, xf=None, flags=None, ws=None, reuse_factors: bool = False):
    """ZF (or regularised, for MMSE) precoding with the uplink estimate from
    symbol 0 of yf and the pilots -> (xf c64 [F][M][D][n_sc], flags).  With
    reuse_factors (16 users), ws is the workspace that csi_detect or
    csi_detect_demod (FP32) just used on the same frames: its factor records
    are reused and the factorisation is skipped."""
    F = _nf(yf)
    D = fr.n_data
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _need(pilots, "pilots", (F, fr.n_sc), torch.complex64)
    _need(sym, "sym", (F, fr.K, D, fr.n_sc), torch.complex64)
    xf = _empty((F, fr.M, D, fr.n_sc), torch.complex64, yf) if xf is None else xf
    flags = _empty((F, fr.n_sc), torch.uint8, yf) if flags is None else flags
    _need(xf, "xf", (F, fr.M, D, fr.n_sc), torch.complex64)
    _need(flags, "flags", (F, fr.n_sc), torch.uint8)
    need = workspace_bytes(fr, F, WS_PRECODE, "fp32")
    if reuse_factors and ws is None:
        raise RxphyError("reuse_factors needs the workspace that holds the uplink's factor records")
    if need and ws is None:
        ws = _empty((need,), torch.uint8, yf)
    _check(load().rxphy_precode(ctypes.byref(fr.c()), F, _ptr(yf), _ptr(pilots), _ptr(sym), _ptr(xf),
                                _ptr(flags), _ptr(ws), ws.numel() if ws is not None else 0,
                                PRECODE_REUSE_FACTORS if reuse_factors else 0, _stream()),
           "rxphy_precode")
    return xf, flags


def modulate_precode(fr: Frame, yf, pilots, bits, xf=None, flags=None, ws=None, reuse_factors: bool = False):
    """modulate then precode in one call (the symbols never stored) ->
    (xf, flags), the same as precode(fr, yf, pilots, modulate(fr, bits))."""
    F = _nf(yf)
    D = fr.n_data
    _need(yf, "yf", (F, fr.M, fr.n_sym, fr.n_sc), torch.complex64)
    _need(pilots, "pilots", (F, fr.n_sc), torch.complex64)
    _need(bits, "bits", (F, fr.K, D, fr.n_sc, fr.qam_bits), torch.uint8)
    xf = _empty((F, fr.M, D, fr.n_sc), torch.complex64, yf) if xf is None else xf
    flags = _empty((F, fr.n_sc), torch.uint8, yf) if flags is None else flags
    _need(xf, "xf", (F, fr.M, D, fr.n_sc), torch.complex64)
    _need(flags, "flags", (F, fr.n_sc), torch.uint8)
    need = workspace_bytes(fr, F, WS_PRECODE, "fp32")
    if reuse_factors and ws is None:
        raise RxphyError("reuse_factors needs the workspace that holds the uplink's factor records")
    if need and ws is None:
        ws = _empty((need,), torch.uint8, yf)
    _check(load().rxphy_modulate_precode(ctypes.byref(fr.c()), F, _ptr(yf), _ptr(pilots), _ptr(bits), _ptr(xf),
                                         _ptr(flags), _ptr(ws), ws.numel() if ws is not None else 0,
                                         PRECODE_REUSE_FACTORS if reuse_factors else 0, _stream()),
           "rxphy_modulate_precode")
    return xf, flags


def ifft(fr: Frame, xf, x=None):
    """Rows of n_sc used subcarriers [..., n_sc] -> time rows [..., cp_len + n_fft]
    (unscaled inverse of fft(), cyclic prefix = the last cp_len samples)."""
    if xf.device.type != "cuda" or xf.dtype != torch.complex64 or not xf.is_contiguous() or xf.shape[-1] != fr.n_sc:
        raise RxphyError("xf: need a contiguous complex64 device tensor [..., %d]" % fr.n_sc)
    rows = xf.numel() // fr.n_sc
    shape = tuple(xf.shape[:-1]) + (fr.cp_len + fr.n_fft,)
    x = _empty(shape, torch.complex64, xf) if x is None else x
    _need(x, "x", shape, torch.complex64)
    _check(load().rxphy_ifft(ctypes.byref(fr.c()), rows, _ptr(xf), _ptr(x), _stream()), "rxphy_ifft")
    return x



def ifft_sc16(fr: Frame, xf, scale: float, x=None):
    """Rows of n_sc used subcarriers [..., n_sc] -> 16-bit I/Q time rows
    [..., cp_len + n_fft, 2] (round(value / scale), saturated)."""
    if xf.device.type != "cuda" or xf.dtype != torch.complex64 or not xf.is_contiguous() or xf.shape[-1] != fr.n_sc:
        raise RxphyError("xf must be a contiguous complex64 device tensor [..., n_sc]")
    shape = tuple(xf.shape[:-1]) + (fr.cp_len + fr.n_fft, 2)
    x = _empty(shape, torch.int16, xf) if x is None else x
    _need(x, "x", shape, torch.int16)
    _check(load().rxphy_ifft_sc16(ctypes.byref(fr.c()), xf.numel() // fr.n_sc, _ptr(xf), float(scale), _ptr(x),
                                  _stream()), "rxphy_ifft_sc16")
    return x

def demod(fr: Frame, xt, nu, llr=None):
    """-> llr f32 [F][K][D][n_sc][qam_bits]."""
    F = _nf(xt)
    D = fr.n_data
    _need(xt, "xt", (F, fr.K, D, fr.n_sc), torch.complex64)
    _need(nu, "nu", (F, fr.K, fr.n_sc), torch.float32)
    if llr is None:
        llr = _empty((F, fr.K, D, fr.n_sc, fr.qam_bits), torch.float32, xt)
    _need(llr, "llr", (F, fr.K, D, fr.n_sc, fr.qam_bits), torch.float32)
    _check(load().rxphy_demod(ctypes.byref(fr.c()), F, _ptr(xt), _ptr(nu), _ptr(llr), _stream()),
           "rxphy_demod")
    return llr


def forward(fr: Frame, x, pilots, precision: str = "fp32", cond_threshold: float = 1e3,
            fused: bool = False):
    """All four stages; returns a dict of every intermediate (no "h" when the
    csi, detect and demod stages run fused)."""
    yf = fft(fr, x)
    if fused:
        llr, nu, flags, xt = csi_detect_demod(fr, yf, pilots, precision, cond_threshold, want_xt=True)
        return dict(yf=yf, xt=xt, nu=nu, flags=flags, llr=llr)
    h = csi(fr, yf, pilots)
    xt, nu, flags = detect(fr, h, yf, precision, cond_threshold)
    llr = demod(fr, xt, nu)
    return dict(yf=yf, h=h, xt=xt, nu=nu, flags=flags, llr=llr)


def backward(fr: Frame, x, pilots, dllr, saved=None, want_dh: bool = False):
    """Adjoint of forward(): dL/dllr -> dL/dx (and dL/dh if asked)."""
    F = _nf(x)
    _need(x, "x", (F, fr.M, fr.n_sym, fr.cp_len + fr.n_fft), torch.complex64)
    _need(pilots, "pilots", (F, fr.n_sc), torch.complex64)
    _need(dllr, "dllr", (F, fr.K, fr.n_data, fr.n_sc, fr.qam_bits), torch.float32)
    dx = torch.empty_like(x)
    dh = _empty((F, fr.M, fr.K, fr.n_sc), torch.complex64, x) if want_dh else None
    sv = None
    if saved is not None:
        sv = _Saved(*[saved[k].data_ptr() if saved.get(k) is not None else None for k in ("yf", "h", "xt", "nu")])
    need = workspace_bytes(fr, F, WS_BACKWARD)
    ws = _empty((max(need, 1),), torch.uint8, x)
    _check(load().rxphy_backward(ctypes.byref(fr.c()), F, _ptr(x), _ptr(pilots),
                                 ctypes.byref(sv) if sv is not None else None, _ptr(dllr),
                                 _ptr(dx), _ptr(dh), _ptr(ws), need, _stream()),
           "rxphy_backward")
    return (dx, dh) if want_dh else dx


class RxphyFunction(torch.autograd.Function):
    """llr = RxphyFunction.apply(x, pilots, frame): the FP32 forward chain with
    the hand-written adjoint of librxphy as its backward (gradient w.r.t. x)."""

    @staticmethod
    def forward(ctx, x, pilots, fr):
        out = forward(fr, x.detach(), pilots)
        ctx.fr = fr
        ctx.save_for_backward(x.detach(), pilots, out["yf"], out["h"], out["xt"], out["nu"])
        return out["llr"]

    @staticmethod
    def backward(ctx, dllr):
        x, pilots, yf, h, xt, nu = ctx.saved_tensors
        dx = backward(ctx.fr, x, pilots, dllr.contiguous(), saved=dict(yf=yf, h=h, xt=xt, nu=nu))
        return dx, None, None


# ------------------------------------------------------------ batched plans
STAGE_FFT, STAGE_CSI, STAGE_DETECT, STAGE_DEMOD, STAGE_ALL = 1, 2, 4, 8, 15
PLAN_WAIT_TIMEOUT = 1


@dataclasses.dataclass(frozen=True)
class Tiles:
    """Work-item sizes of one frame in a plan (0 = the library default)."""
    fft_iters: int = 0
    csi_tiles: int = 0
    det_tiles: int = 0
    det_kp: int = 0
    dem_groups: int = 0

    def c(self) -> _Tiles:
        return _Tiles(self.fft_iters, self.csi_tiles, self.det_tiles, self.det_kp, self.dem_groups)


class Plan:
    """Frames of differing shape run by one persistent launch (rxphy_plan_*).

    Buffers are packed byte tensors (one per tensor name in ``TENSORS``);
    ``view(bufs, name, f)`` is frame f's tensor inside them, shaped as the
    single-frame calls shape it with F = 1."""

    TENSORS = _TENSORS

    def __init__(self, frames, tiles=None, stages: int = 0, grid: int = 0, spin_limit: int = 0,
                 fuse_csi: bool = False, fuse_demod: bool = False):
        lib = load()
        self.frames = list(frames)
        n = len(self.frames)
        arr = (_Frame * n)(*[f.c() for f in self.frames])
        if tiles is None:
            tarr = None
        else:
            tl = list(tiles) if isinstance(tiles, (list, tuple)) else [tiles] * n
            if len(tl) != n:
                raise RxphyError("tiles needs one entry per frame")
            tarr = (_Tiles * n)(*[t.c() for t in tl])
        opt = _PlanOptions(int(stages), int(grid), int(spin_limit), 1 if fuse_csi else 0, 1 if fuse_demod else 0)
        self.fuse_csi = bool(fuse_csi)
        self.fuse_demod = bool(fuse_demod)
        h = ctypes.c_void_p()
        _check(lib.rxphy_plan_create(arr, n, tarr, ctypes.byref(opt), ctypes.byref(h)),
               "rxphy_plan_create")
        self._h = h
        offs = (_Offsets * n)()
        tot = _Offsets()
        _check(lib.rxphy_plan_layout(h, offs, ctypes.byref(tot)), "rxphy_plan_layout")
        self.offsets = [{k: int(getattr(o, k)) for k in _TENSORS} for o in offs]
        self.totals = {k: int(getattr(tot, k)) for k in _TENSORS}
        counts = (ctypes.c_int64 * 4)()
        g = ctypes.c_int32()
        _check(lib.rxphy_plan_info(h, counts, ctypes.byref(g)), "rxphy_plan_info")
        self.counts = [int(c) for c in counts]
        self.grid = int(g.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rxphy_plan_destroy(h)
            self._h = None

    # ---- buffers
    def shape(self, name: str, f: int):
        fr = self.frames[f]
        return {"x": (fr.M, fr.n_sym, fr.cp_len + fr.n_fft), "pilots": (fr.n_sc,),
                "yf": (fr.M, fr.n_sym, fr.n_sc), "h": (fr.M, fr.K, fr.n_sc),
                "xt": (fr.K, fr.n_data, fr.n_sc), "nu": (fr.K, fr.n_sc), "flags": (fr.n_sc,),
                "llr": (fr.K, fr.n_data, fr.n_sc, fr.qam_bits)}[name]

    @staticmethod
    def dtype(name: str):
        return {"x": torch.complex64, "pilots": torch.complex64, "yf": torch.complex64,
                "h": torch.complex64, "xt": torch.complex64, "nu": torch.float32,
                "flags": torch.uint8, "llr": torch.float32}[name]

    def _placeholder(self, k: str) -> bool:
        """h is never written when the plan fuses the CSI stage into the
        detector, x_tilde never when it fuses the demod stage in."""
        return (k == "h" and self.fuse_csi) or (k == "xt" and self.fuse_demod)

    def alloc(self, device="cuda"):
        """One packed byte buffer per tensor (a one-byte placeholder for a
        tensor the plan never writes)."""
        return {k: torch.empty((1 if self._placeholder(k) else max(self.totals[k], 1),),
                               dtype=torch.uint8, device=device) for k in _TENSORS}

    def view(self, bufs, name: str, f: int):
        shp = self.shape(name, f)
        dt = self.dtype(name)
        n = 1
        for d in shp:
            n *= d
        nbytes = n * torch.empty((), dtype=dt).element_size()
        o = self.offsets[f][name]
        return bufs[name][o:o + nbytes].view(dt).view(shp)

    def _batch(self, bufs) -> _Batch:
        for k in _TENSORS:
            t = bufs[k]
            need = 1 if self._placeholder(k) else self.totals[k]
            if t.device.type != "cuda" or t.numel() * t.element_size() < need:
                raise RxphyError("buffer %s must be a device tensor of >= %d bytes" % (k, need))
        return _Batch(*[bufs[k].data_ptr() for k in _TENSORS])

    # ---- runs
    def forward(self, bufs):
        b = self._batch(bufs)
        _check(load().rxphy_plan_forward(self._h, ctypes.byref(b), _stream()), "rxphy_plan_forward")

    def graph(self, bufs):
        b = self._batch(bufs)
        _check(load().rxphy_plan_graph(self._h, ctypes.byref(b)), "rxphy_plan_graph")
        self._graph_bufs = bufs      # keep the bound buffers alive

    def replay(self):
        _check(load().rxphy_plan_replay(self._h, _stream()), "rxphy_plan_replay")

    def device_status(self) -> int:
        v = ctypes.c_uint32()
        _check(load().rxphy_plan_device_status(self._h, ctypes.byref(v)), "rxphy_plan_device_status")
        return int(v.value)


# ------------------------------------------------------------------ streaming
def clock_ns() -> int:
    """The steady clock the streaming runtime stamps completions with."""
    return int(load().rxphy_clock_ns())


def latency_summary(lat_us, bound_us: float) -> dict:
    """Nearest-rank p50 / p99 / max / mean of latencies (microseconds), the
    count within bound_us, and whether at least 99 % met it."""
    a = np.ascontiguousarray(np.asarray(lat_us, dtype=np.float64))
    out = _LatencySummary()
    _check(load().rxphy_latency_summarize(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size,
                                          float(bound_us), ctypes.byref(out)), "rxphy_latency_summarize")
    return {k: getattr(out, k) for k, _ in _LatencySummary._fields_}


def _host_array(addr: int, shape, dtype):
    n = int(np.prod(shape)) * np.dtype(dtype).itemsize
    buf = (ctypes.c_uint8 * n).from_address(addr)
    return np.frombuffer(buf, dtype=dtype).reshape(shape)


class Stream:
    """Real-time task stream (rxphy_stream_*): ``depth`` slots handed out in
    turn, a task = fft + fused csi/detect/demod over ``n_frames`` frames.

    host_io=True: ``host(slot)`` gives numpy views of the slot's pinned host
    buffers (x, pilots in; llr, nu, flags out), valid until ``close()``.
    sc16_scale > 0: the samples are 16-bit I/Q pairs (as ``fft_sc16``).
    host_io=False: ``submit`` takes device tensors for the task's inputs and
    outputs; the task runs on the slot's own HIP stream, so the inputs must
    already be complete (synchronise their producer first), and the outputs
    are complete after ``drain()``."""

    def __init__(self, fr: Frame, n_frames: int, depth: int = 2, host_io: bool = True, sc16_scale: float = 0.0):
        lib = load()
        self.fr, self.nf, self.depth, self.host_io = fr, int(n_frames), int(depth), bool(host_io)
        self.sc16 = float(sc16_scale)
        h = ctypes.c_void_p()
        _check(lib.rxphy_stream_create(ctypes.byref(fr.c()), self.nf, self.depth, int(self.host_io),
                                       self.sc16, ctypes.byref(h)), "rxphy_stream_create")
        self._h = h
        self._keep = {}

    def shapes(self):
        fr, F = self.fr, self.nf
        xs = ((F, fr.M, fr.n_sym, fr.cp_len + fr.n_fft, 2), np.int16) if self.sc16 > 0 else \
            ((F, fr.M, fr.n_sym, fr.cp_len + fr.n_fft), np.complex64)
        return {"x": xs,
                "pilots": ((F, fr.n_sc), np.complex64),
                "llr": ((F, fr.K, fr.n_data, fr.n_sc, fr.qam_bits), np.float32),
                "nu": ((F, fr.K, fr.n_sc), np.float32), "flags": ((F, fr.n_sc), np.uint8)}

    def host(self, slot: int) -> dict:
        hb = _StreamHost()
        _check(load().rxphy_stream_host_buffers(self._h, int(slot), ctypes.byref(hb)),
               "rxphy_stream_host_buffers")
        return {k: _host_array(getattr(hb, k), shp, dt) for k, (shp, dt) in self.shapes().items()}

    def acquire(self) -> int:
        v = ctypes.c_int32()
        _check(load().rxphy_stream_acquire(self._h, ctypes.byref(v)), "rxphy_stream_acquire")
        return int(v.value)

    def submit(self, slot: int, arrival_ns: int = 0, x=None, pilots=None, llr=None, nu=None, flags=None):
        if not self.host_io:
            shp = self.shapes()
            for name, t, dt in (("x", x, torch.int16 if self.sc16 > 0 else torch.complex64),
                                ("pilots", pilots, torch.complex64),
                                ("llr", llr, torch.float32), ("nu", nu, torch.float32)):
                if t is None:
                    raise RxphyError("device-resident stream: %s is required" % name)
                _need(t, name, shp[name][0], dt)
            if flags is not None:
                _need(flags, "flags", shp["flags"][0], torch.uint8)
            self._keep[int(slot)] = (x, pilots, llr, nu, flags)
        _check(load().rxphy_stream_submit(self._h, int(slot), int(arrival_ns), _ptr(x), _ptr(pilots),
                                          _ptr(llr), _ptr(nu), _ptr(flags)), "rxphy_stream_submit")

    def drain(self):
        _check(load().rxphy_stream_drain(self._h), "rxphy_stream_drain")

    def latencies(self) -> np.ndarray:
        n = ctypes.c_int64()
        lib = load()
        _check(lib.rxphy_stream_latencies(self._h, None, 0, ctypes.byref(n)), "rxphy_stream_latencies")
        out = np.empty(n.value, dtype=np.float64)
        _check(lib.rxphy_stream_latencies(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          out.size, ctypes.byref(n)), "rxphy_stream_latencies")
        return out

    def reset_latencies(self):
        _check(load().rxphy_stream_reset_latencies(self._h), "rxphy_stream_reset_latencies")

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rxphy_stream_destroy(h)
        self._h = None
        self._keep = {}

    def __del__(self):
        self.close()


# ------------------------------------------------------------------- sensing
@dataclasses.dataclass(frozen=True)
class SenseConfig:
    """Spectrum-sensing configuration (mirrors ``rxphy_sense_config``)."""
    n_fft: int = 1024
    n_rows: int = 2000
    sg_window: int = 21
    sg_order: int = 1
    psd_factor: float = 1.1
    bins: int = 256

    def c(self) -> _SenseConfig:
        return _SenseConfig(self.n_fft, self.n_rows, self.sg_window, self.sg_order, self.psd_factor, self.bins)


def sense_workspace_bytes(cfg: SenseConfig, n_plots: int) -> int:
    return int(load().rxphy_sense_workspace_bytes(ctypes.byref(cfg.c()), int(n_plots)))


def sense(cfg: SenseConfig, x, max_boxes: int = 1024, intermediates: bool = False, ws=None, boxes=None,
          n_boxes=None) -> dict:
    """x c64 [P][T][F] -> dict(n_boxes i32 [P], boxes i32 [P][max_boxes][4]
    (t0, f0, t1, f1); with intermediates: tf, psd, psd_smooth, floor,
    otsu_bin, mask, mask_mo)."""
    P = _nf(x)
    T, F = cfg.n_rows, cfg.n_fft
    _need(x, "x", (P, T, F), torch.complex64)
    dev = x.device
    out = {}
    if intermediates:
        out = {"tf": torch.empty((P, T, F), dtype=torch.float32, device=dev),
               "psd": torch.empty((P, F), dtype=torch.float32, device=dev),
               "psd_smooth": torch.empty((P, F), dtype=torch.float32, device=dev),
               "floor": torch.empty((P, 2), dtype=torch.float32, device=dev),
               "otsu_bin": torch.empty((P, F), dtype=torch.int32, device=dev),
               "mask": torch.empty((P, T, F), dtype=torch.uint8, device=dev),
               "mask_mo": torch.empty((P, T, F), dtype=torch.uint8, device=dev)}
    o = _SenseOutputs(*[out[k].data_ptr() if k in out else None for k in _SENSE_OUT])
    n_boxes = torch.empty((P,), dtype=torch.int32, device=dev) if n_boxes is None else n_boxes
    _need(n_boxes, "n_boxes", (P,), torch.int32)
    if boxes is None:
        boxes = torch.empty((P, max(max_boxes, 0), 4), dtype=torch.int32, device=dev)
    _need(boxes, "boxes", (P, max_boxes, 4), torch.int32)
    need = sense_workspace_bytes(cfg, P)
    if need == 0:
        raise RxphyError("invalid sense config %s" % (cfg,))
    if ws is None or ws.numel() < need:
        ws = torch.empty((need,), dtype=torch.uint8, device=dev)
    _check(load().rxphy_sense(ctypes.byref(cfg.c()), P, _ptr(x), ctypes.byref(o), _ptr(n_boxes),
                              _ptr(boxes) if max_boxes > 0 else None, int(max_boxes), _ptr(ws), ws.numel(),
                              _stream()), "rxphy_sense")
    out.update(n_boxes=n_boxes, boxes=boxes)
    return out


def savgol_weights(window: int, order: int) -> np.ndarray:
    """The Savitzky-Golay weights the sensing pipeline smooths the PSD with
    (float32, `window` values, offsets -window/2 .. window/2); host only."""
    w = np.zeros(int(window), dtype=np.float32)
    _check(load().rxphy_savgol_weights(int(window), int(order), w.ctypes.data), "rxphy_savgol_weights")
    return w


def box_metrics(gt, det, theta_iou: float, want_iou: bool = False) -> dict:
    """Section III-A detection metrics of inclusive (t0, f0, t1, f1) boxes."""
    g = np.ascontiguousarray(np.asarray(gt, dtype=np.int32).reshape(-1, 4))
    d = np.ascontiguousarray(np.asarray(det, dtype=np.int32).reshape(-1, 4))
    iou = np.zeros((len(g), len(d)), dtype=np.float64) if want_iou else None
    m = _Metrics()
    _check(load().rxphy_box_metrics(g.ctypes.data if len(g) else None, len(g), d.ctypes.data if len(d) else None,
                                    len(d), float(theta_iou), iou.ctypes.data if want_iou and iou.size else None,
                                    ctypes.byref(m)), "rxphy_box_metrics")
    r = {k: getattr(m, k) for k, _ in _Metrics._fields_}
    if want_iou:
        r["iou"] = iou
    return r


# ------------------------------------------------------------------ LDPC decoding
class LdpcCode:
    """A quasi-cyclic LDPC code from its base matrix (int16 [mb][nb]: -1 = zero
    block, s = identity cyclically shifted by s) and lifting size z; owns the
    device edge table of rxphy_ldpc_code_create."""

    def __init__(self, base, z: int):
        lib = load()
        b = np.ascontiguousarray(np.asarray(base, dtype=np.int16))
        if b.ndim != 2:
            raise RxphyError("base must be a 2-D matrix")
        self.base = b
        self.mb, self.nb = b.shape
        self.z = int(z)
        self.n = self.nb * self.z
        h = ctypes.c_void_p()
        _check(lib.rxphy_ldpc_code_create(b.ctypes.data, self.mb, self.nb, self.z, ctypes.byref(h)),
               "rxphy_ldpc_code_create")
        self._h = h

    def workspace_bytes(self, n_cw: int) -> int:
        return int(load().rxphy_ldpc_workspace_bytes(self._h, int(n_cw)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rxphy_ldpc_code_destroy(h)
            self._h = None


def ldpc_decode(code: LdpcCode, llr, max_iter: int = 10, alpha: float = 0.75, post=None, bits=None,
                iters=None, ws=None):
    """llr f32 [n_cw][N] -> (posterior LLRs f32 [n_cw][N], hard bits u8
    [n_cw][N], iterations i32 [n_cw])."""
    n_cw = _nf(llr)
    _need(llr, "llr", (n_cw, code.n), torch.float32)
    post = _empty((n_cw, code.n), torch.float32, llr) if post is None else post
    bits = _empty((n_cw, code.n), torch.uint8, llr) if bits is None else bits
    iters = _empty((n_cw,), torch.int32, llr) if iters is None else iters
    _need(post, "post", (n_cw, code.n), torch.float32)
    _need(bits, "bits", (n_cw, code.n), torch.uint8)
    _need(iters, "iters", (n_cw,), torch.int32)
    need = code.workspace_bytes(n_cw)
    if ws is None:
        ws = _empty((max(need, 4),), torch.uint8, llr)
    _check(load().rxphy_ldpc_decode(code._h, n_cw, _ptr(llr), int(max_iter), float(alpha), _ptr(post), _ptr(bits),
                                    _ptr(iters), _ptr(ws), ws.numel(), _stream()), "rxphy_ldpc_decode")
    return post, bits, iters
