"""GPU checks of the 16-bit I/Q ingest (rxphy_fft_sc16, the fronthaul format
of Section IV-D): with a power-of-two scale the converted samples are exact,
so the transform equals rxphy_fft of the converted complex64 samples bit for
bit; with any other scale it matches the FP64 oracle within the FFT
tolerance; a stream of 16-bit tasks returns what the direct calls return."""
import numpy as np
import pytest

import oracle as O
import synth
from parity_util import rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-sc16]", *a, flush=True)


def to_c64(q, scale):
    return (q[..., 0].astype(np.float32) * np.float32(scale)
            + 1j * (q[..., 1].astype(np.float32) * np.float32(scale))).astype(np.complex64)


SHAPES = [synth.config_shape(2), synth.config_shape(1), synth.Shape(8, 4, 1024, 601, 5, 72, 4),
          synth.Shape(4, 2, 4096, 3276, 3, 288, 6)]


@pytest.mark.parametrize("sh", SHAPES)
def test_sc16_equals_fft_of_converted_samples(rx, sh):
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    rng = np.random.default_rng([31, sh.n_fft, sh.M])
    q = rng.integers(-32768, 32768, (2, sh.M, sh.n_sym, sh.cp_len + sh.n_fft, 2)).astype(np.int16)
    for scale in (1.0, 2.0 ** -12, 2.0 ** 5):
        y16 = rx.fft_sc16(fr, torch.from_numpy(q).cuda(), scale)
        y32 = rx.fft(fr, torch.from_numpy(to_c64(q, scale)).cuda())
        torch.cuda.synchronize()
        assert torch.equal(y16, y32), (sh, scale)
    scale = 0.3                                        # not a power of two: rounded on conversion
    y = rx.fft_sc16(fr, torch.from_numpy(q).cuda(), scale).cpu().numpy()
    xs = q[..., 0].astype(np.float64) * scale + 1j * q[..., 1].astype(np.float64) * scale
    ref = O.fft_stage(xs, sh.n_fft, sh.n_sc, sh.cp_len)
    e = rel_rms(y, ref)
    say(sh, "scale 0.3 rel_rms", e)
    assert e < 2e-6


def test_quantised_headline_frames_through_the_chain(rx):
    """Headline frames quantised to 16 bits: the 16-bit chain equals the
    complex64 chain on the dequantised samples bit for bit, and the hard bits
    of the unquantised frames change only inside the quantisation noise."""
    sh = synth.config_shape(2)
    frs = [synth.make_frame(2, f) for f in range(3)]
    x = np.stack([f.x for f in frs])
    q, scale = synth.quantize_sc16(x)
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    p = torch.from_numpy(np.stack([f.pilots for f in frs])).cuda()
    llr16, nu16, fl16, _ = rx.csi_detect_demod(fr, rx.fft_sc16(fr, torch.from_numpy(q).cuda(), scale), p)
    llrq, nuq, flq, _ = rx.csi_detect_demod(fr, rx.fft(fr, torch.from_numpy(to_c64(q, scale)).cuda()), p)
    llr, _, _, _ = rx.csi_detect_demod(fr, rx.fft(fr, torch.from_numpy(x).cuda()), p)
    torch.cuda.synchronize()
    assert torch.equal(llr16, llrq) and torch.equal(nu16, nuq) and torch.equal(fl16, flq)
    a, b = llr16.cpu().numpy(), llr.cpu().numpy()
    rms = np.sqrt(np.mean(b ** 2))
    flips = int(np.sum((a < 0) != (b < 0)))
    say("scale", scale, "hard-bit flips vs unquantised", flips, "of", b.size,
        "max |dLLR| / rms", float(np.max(np.abs(a - b)) / rms))
    assert flips <= 1e-4 * b.size


def test_sc16_stream_equals_direct_calls(rx):
    sh = synth.config_shape(2)
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    st = rx.Stream(fr, 2, depth=2, host_io=True, sc16_scale=2.0 ** -6)
    try:
        refs = {}
        for task in range(2):
            frs = [synth.make_frame(2, 10 + 2 * task + i) for i in range(2)]
            q, _ = synth.quantize_sc16(np.stack([f.x for f in frs]))
            pil = np.stack([f.pilots for f in frs])
            slot = st.acquire()
            h = st.host(slot)
            h["x"][...] = q
            h["pilots"][...] = pil
            st.submit(slot)
            pd = torch.from_numpy(pil).cuda()
            l, n, f, _ = rx.csi_detect_demod(fr, rx.fft_sc16(fr, torch.from_numpy(q).cuda(), 2.0 ** -6), pd)
            refs[slot] = (l.cpu().numpy(), n.cpu().numpy(), f.cpu().numpy())
        st.drain()
        for slot, (l, n, f) in refs.items():
            h = st.host(slot)
            assert np.array_equal(h["llr"], l) and np.array_equal(h["nu"], n) and np.array_equal(h["flags"], f)
    finally:
        st.close()


@pytest.mark.parametrize("N,n_sc,cp", [(2048, 1200, 0), (1024, 601, 72), (512, 300, 36)])
def test_ifft_sc16_is_the_quantised_ifft(rx, N, n_sc, cp):
    """The 16-bit inverse output equals the FP32 inverse output multiplied by
    1/scale in FP32, rounded to nearest even and saturated, bit for bit,
    prefix included; a scale that overdrives the range saturates."""
    sh = synth.Shape(4, 2, N, n_sc, 3, cp, 2)
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    rng = np.random.default_rng([33, N])
    X = ((rng.standard_normal((2, 4, 3, n_sc)) + 1j * rng.standard_normal((2, 4, 3, n_sc))) * 3.0).astype(np.complex64)
    xf = torch.from_numpy(X).cuda()
    x32 = rx.ifft(fr, xf).cpu().numpy()
    for scale in (2.0 ** -8, 0.0173, 2.0 ** -14):
        q = rx.ifft_sc16(fr, xf, scale).cpu().numpy()
        s = np.float32(1.0) / np.float32(scale)
        ref = np.stack([np.rint(x32.real.astype(np.float32) * s), np.rint(x32.imag.astype(np.float32) * s)], -1)
        ref = np.clip(ref, -32768, 32767).astype(np.int16)
        sat = int(np.sum(np.abs(ref.astype(np.int32)) >= 32767))
        say("ifft_sc16", N, n_sc, cp, "scale", scale, "saturated", sat)
        assert np.array_equal(q, ref)
        assert np.array_equal(q[..., :cp, :], q[..., N:N + cp, :])
