"""Host-only checks of the streaming runtime: the nearest-rank latency
summary (the bounded-latency rule of Section III-B: at least 99 % of tasks
within the bound) and argument validation before any HIP call."""
import ctypes
import math

import numpy as np
import pytest

import paper_2603_20481_amd as rx


def nearest_rank(v, p):
    s = sorted(v)
    return s[math.ceil(p * len(s) / 100) - 1]


def test_summary_matches_nearest_rank_definition():
    rng = np.random.default_rng(3)
    for n in list(range(1, 40)) + [99, 100, 101, 199, 200, 1000, 1001]:
        lat = rng.gamma(2.0, 100.0, n)
        bound = float(np.quantile(lat, rng.uniform(0.9, 1.0)))
        s = rx.latency_summary(lat, bound)
        assert s["count"] == n
        assert s["p50_us"] == nearest_rank(lat, 50)
        assert s["p99_us"] == nearest_rank(lat, 99)
        assert s["max_us"] == lat.max()
        assert s["mean_us"] == pytest.approx(lat.mean(), rel=1e-12)
        assert s["on_time"] == int(np.sum(lat <= bound))
        # the rule "at least 99 % on time" is exactly "p99 within the bound"
        assert bool(s["meets_99"]) == (100 * s["on_time"] >= 99 * n) == (s["p99_us"] <= bound)


def test_summary_edges():
    lat = np.arange(1, 101, dtype=float)             # 100 tasks, 1 .. 100 us
    s = rx.latency_summary(lat, 99.0)                # one late task: 99 % on time
    assert (s["on_time"], s["meets_99"], s["p99_us"]) == (99, 1, 99.0)
    s = rx.latency_summary(lat, 98.0)                # two late tasks
    assert (s["on_time"], s["meets_99"]) == (98, 0)
    s = rx.latency_summary([5.0], 5.0)               # bound inclusive
    assert (s["count"], s["on_time"], s["meets_99"], s["p99_us"]) == (1, 1, 1, 5.0)
    s = rx.latency_summary([], 1.0)
    assert s["count"] == 0 and s["meets_99"] == 0
    with pytest.raises(rx.RxphyError):
        rx.latency_summary([1.0, float("nan")], 1.0)


@pytest.mark.parametrize("kw", [dict(n_frames=0), dict(n_frames=65536), dict(depth=0), dict(depth=9),
                                dict(host_io=2), dict(sc16=-1.0), dict(sc16=float("nan")),
                                dict(sc16=float("inf"))])
def test_create_rejects_bad_arguments_before_the_gpu(kw):
    a = dict(n_frames=1, depth=2, host_io=1, sc16=0.0)
    a.update(kw)
    fr = rx.Frame(8, 2, 512, 300, 14, 0, 2)
    h = ctypes.c_void_p(1)
    st = rx.load().rxphy_stream_create(ctypes.byref(fr.c()), a["n_frames"], a["depth"], a["host_io"],
                                       a["sc16"], ctypes.byref(h))
    assert st == 1 and not h.value


def test_create_rejects_bad_frames():
    for fr in (rx.Frame(8, 9, 512, 300), rx.Frame(8, 2, 500, 300), rx.Frame(8, 2, 512, 600)):
        with pytest.raises(rx.RxphyError):
            rx.Stream(fr, 1, 2, True)


def test_null_stream_calls_fail_cleanly():
    lib = rx.load()
    v = ctypes.c_int32()
    assert lib.rxphy_stream_acquire(None, ctypes.byref(v)) == 1
    assert lib.rxphy_stream_submit(None, 0, 0, None, None, None, None, None) == 1
    assert lib.rxphy_stream_drain(None) == 1
    assert lib.rxphy_stream_reset_latencies(None) == 1
    n = ctypes.c_int64()
    assert lib.rxphy_stream_latencies(None, None, 0, ctypes.byref(n)) == 1
    lib.rxphy_stream_destroy(None)
    assert rx.clock_ns() > 0


def test_fft_sc16_argument_checks():
    lib = rx.load()
    fr = rx.Frame(8, 2, 512, 300, 14, 0, 2)
    p = ctypes.c_void_p(256)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        assert lib.rxphy_fft_sc16(ctypes.byref(fr.c()), 1, p, bad, p, None) == 1
    assert lib.rxphy_fft_sc16(ctypes.byref(fr.c()), 1, None, 1.0, p, None) == 1
    assert lib.rxphy_fft_sc16(ctypes.byref(fr.c()), 0, None, 1.0, None, None) == 0   # nothing to do


def test_quantizer_is_a_power_of_two_scale():
    import synth
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(1000) + 1j * rng.standard_normal(1000)) * 37.0
    q, scale = synth.quantize_sc16(x)
    assert np.log2(scale) == int(np.log2(scale))
    assert np.abs(q).max() <= 32767 // 2 + 1
    back = q[..., 0] * scale + 1j * q[..., 1] * scale
    assert np.max(np.abs(back - x)) <= scale * 0.5 * np.sqrt(2) + 1e-12


def test_precode_option_checks():
    lib = rx.load()
    p = ctypes.c_void_p(256)
    fr16 = rx.Frame(32, 16, 512, 300, 6, 0, 2)
    fr8 = rx.Frame(32, 8, 512, 300, 6, 0, 2)
    assert lib.rxphy_precode(ctypes.byref(fr16.c()), 1, p, p, p, p, None, p, 1 << 20, 2, None) == 1   # unknown option
    assert lib.rxphy_precode(ctypes.byref(fr8.c()), 1, p, p, p, p, None, None, 0, 1, None) == 1       # reuse needs K = 16
