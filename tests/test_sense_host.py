"""Host-only checks of the sensing entry points: the detection metrics of
Section III-A (rxphy_box_metrics, host code) against the oracle on random
boxes, the Savitzky-Golay weights (rxphy_savgol_weights, host code) against
scipy, and configuration checks made before any HIP call."""
import ctypes

import numpy as np
import pytest

import paper_2603_20481_amd as rx
from oracle import sensing_oracle as S


def random_boxes(rng, n, T=200, F=300):
    t0 = rng.integers(0, T - 1, n)
    f0 = rng.integers(0, F - 1, n)
    t1 = np.minimum(T - 1, t0 + rng.integers(0, 40, n))
    f1 = np.minimum(F - 1, f0 + rng.integers(0, 60, n))
    return np.stack([t0, f0, t1, f1], axis=1).astype(np.int32)


def test_metrics_match_oracle():
    rng = np.random.default_rng(12)
    for trial in range(60):
        gt = random_boxes(rng, int(rng.integers(0, 8)))
        k = int(rng.integers(0, len(gt) + 1))
        near = gt[:k] + rng.integers(-3, 4, (k, 4))          # detections close to ground truths
        near[:, 2] = np.maximum(near[:, 2], near[:, 0])
        near[:, 3] = np.maximum(near[:, 3], near[:, 1])
        det = np.concatenate([near, random_boxes(rng, int(rng.integers(0, 6)))]).astype(np.int32)
        for theta in (0.0, 0.3, 0.5, 0.9):
            a = rx.box_metrics(gt, det, theta, want_iou=True)
            b = S.metrics(gt, det, theta)
            assert (a["n_t"], a["n_f"]) == (b["n_t"], b["n_f"])
            for k in ("p_d", "p_fa", "mean_iou"):
                assert (np.isnan(a[k]) and np.isnan(b[k])) or a[k] == pytest.approx(b[k], rel=1e-12), k
            assert np.allclose(a["iou"], b["iou"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("bad", [dict(n_fft=768), dict(n_rows=2), dict(n_rows=4097), dict(sg_window=20),
                                 dict(sg_window=65), dict(sg_order=7), dict(sg_window=5, sg_order=5),
                                 dict(psd_factor=0.0), dict(psd_factor=float("nan")), dict(bins=1),
                                 dict(bins=257)])
def test_bad_configs_rejected_before_the_gpu(bad):
    cfg = rx.SenseConfig(**{**dict(n_fft=512, n_rows=100), **bad})
    assert rx.sense_workspace_bytes(cfg, 1) == 0
    lib = rx.load()
    n = ctypes.c_int32()
    st = lib.rxphy_sense(ctypes.byref(cfg.c()), 1, ctypes.c_void_p(16), None, ctypes.byref(n), None, 0,
                         None, 0, None)
    assert st == 1


def test_argument_checks():
    lib = rx.load()
    cfg = rx.SenseConfig(n_fft=512, n_rows=100)
    need = rx.sense_workspace_bytes(cfg, 2)
    assert need > 2 * 100 * 512 * 4
    p = ctypes.c_void_p(256)
    n = ctypes.c_void_p(512)
    c = ctypes.byref(cfg.c())
    assert lib.rxphy_sense(c, 0, p, None, n, None, 0, p, need, None) == 1          # no plots
    assert lib.rxphy_sense(c, 2, None, None, n, None, 0, p, need, None) == 1       # no input
    assert lib.rxphy_sense(c, 2, p, None, n, None, 4, p, need, None) == 1          # boxes missing
    assert lib.rxphy_sense(c, 2, p, None, n, p, -1, p, need, None) == 1            # negative max
    assert lib.rxphy_sense(c, 2, p, None, n, p, 4, p, need - 1, None) == 3         # small workspace
    assert lib.rxphy_sense(c, 2, p, None, n, p, 4, ctypes.c_void_p(384), need, None) == 3   # misaligned
    assert lib.rxphy_box_metrics(None, 1, None, 0, 0.5, None, None) == 1


@pytest.mark.parametrize("window,order", [(3, 0), (5, 2), (21, 1), (21, 3), (31, 6), (63, 4), (63, 6), (7, 6)])
def test_savgol_weights_match_scipy(window, order):
    """The host routine (scaled normal equations, Gaussian elimination with
    partial pivoting in FP64, rounded to FP32) against scipy's least-squares
    Savitzky-Golay coefficients."""
    signal = pytest.importorskip("scipy.signal")
    w = rx.savgol_weights(window, order)
    ref = signal.savgol_coeffs(window, order)
    assert w.dtype == np.float32 and w.shape == (window,)
    assert np.max(np.abs(w - ref)) <= 4e-7 * np.max(np.abs(ref)) + 1e-9
    assert abs(float(np.sum(w.astype(np.float64))) - 1.0) < 1e-5        # reproduces constants


@pytest.mark.parametrize("window,order", [(2, 0), (4, 1), (65, 2), (5, 7), (5, 5), (5, -1), (1, 0)])
def test_savgol_weights_argument_checks(window, order):
    with pytest.raises(rx.RxphyError):
        rx.savgol_weights(window, order)
