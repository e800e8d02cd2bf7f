"""GPU parity of the downlink stages (QAM mapping, zero-forcing precoder with
the uplink estimate, inverse transform with a cyclic prefix) against the FP64
oracle, through the C ABI."""
import numpy as np
import pytest

import oracle as O
import synth
from parity_util import rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-downlink]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("q", [2, 4, 6])
def test_modulate_vs_oracle(rx, q):
    sh = synth.Shape(8, 5, 512, 300, 6, 0, q)
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    rng = np.random.default_rng([21, q])
    bits = rng.integers(0, 2, (2, sh.K, sh.n_data, sh.n_sc, q)).astype(np.uint8)
    s = host(rx.modulate(fr, dev(bits)))
    ref = O.modulate_stage(bits, q)
    err = float(np.max(np.abs(s - ref)))
    say("modulate", q, "max abs error", err)
    # FP32 levels: a few units in the last place at magnitude <= 7/sqrt(42)
    assert err < 4 * 2.0 ** -23


@pytest.mark.parametrize("q", [2, 4, 6])
@pytest.mark.parametrize("boff,soff", [(0, 0), (1, 0), (0, 1), (2, 3)])
def test_modulate_ragged_and_misaligned(rx, q, boff, soff):
    """A point count that is not a multiple of four (the ragged tail) and bits
    or symbols that start off their word / 16-byte boundary (the byte path)
    give the same points as the oracle."""
    sh = synth.Shape(4, 3, 512, 301, 2, 0, q)
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    rng = np.random.default_rng([23, q, boff, soff])
    bits = rng.integers(0, 2, (1, sh.K, sh.n_data, sh.n_sc, q)).astype(np.uint8)
    bits[0, 0, 0, :5] *= 7                                   # non-zero bytes other than 1 are ones
    n = bits.size
    bbuf = torch.zeros(n + 8, dtype=torch.uint8, device="cuda")
    bbuf[boff:boff + n] = dev(bits.reshape(-1))
    sbuf = torch.full((sh.K * sh.n_sc + 8,), complex(9.0, 9.0), dtype=torch.complex64, device="cuda")
    sym = sbuf[soff:soff + sh.K * sh.n_sc].view(1, sh.K, 1, sh.n_sc)
    rx.modulate(fr, bbuf[boff:boff + n].view(bits.shape), sym)
    ref = O.modulate_stage((bits != 0).astype(np.uint8), q)
    err = float(np.max(np.abs(host(sym) - ref)))
    say("modulate ragged", q, boff, soff, "points", sh.K * sh.n_sc, "max abs error", err)
    assert err < 4 * 2.0 ** -23
    rest = host(sbuf)
    assert np.all(rest[:soff] == 9 + 9j) and np.all(rest[soff + sh.K * sh.n_sc:] == 9 + 9j)


@pytest.mark.parametrize("N,n_sc,cp", [(512, 300, 36), (2048, 1200, 0), (4096, 3276, 288), (1024, 601, 7)])
def test_ifft_vs_oracle_prefix_and_round_trip(rx, N, n_sc, cp):
    sh = synth.Shape(4, 2, N, n_sc, 3, cp, 2)
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    rng = np.random.default_rng([22, N])
    X = (rng.standard_normal((2, 4, 3, n_sc)) + 1j * rng.standard_normal((2, 4, 3, n_sc))).astype(np.complex64)
    x = rx.ifft(fr, dev(X))
    xh = host(x)
    ref = O.ifft_stage(X, N, n_sc, cp)
    e = rel_rms(xh, ref)
    say("ifft", N, n_sc, cp, "rel_rms", e)
    assert e < 2e-6
    assert np.array_equal(xh[..., :cp], xh[..., N:N + cp])          # prefix = tail, copied
    back = host(rx.fft(fr, x.reshape(2, 4, 3, cp + N)))
    e2 = rel_rms(back, N * X.astype(np.complex128))
    say("  fft(ifft(X)) vs N X rel_rms", e2)
    assert e2 < 2e-6


PRECODE_CASES = [(synth.Shape(64, 16, 2048, 1200, 14, 0, 4), O.ZF),
                 (synth.Shape(64, 16, 2048, 1200, 14, 0, 4), O.MMSE),
                 (synth.Shape(21, 16, 512, 500, 17, 0, 2), O.ZF),
                 (synth.Shape(16, 16, 512, 200, 6, 8, 6), O.MMSE),
                 (synth.Shape(64, 16, 4096, 3276, 17, 0, 6), O.ZF),
                 # fewer than 16 users: one wave per pilot group of K subcarriers
                 (synth.Shape(32, 8, 1024, 600, 14, 0, 4), O.ZF),
                 (synth.Shape(32, 8, 1024, 600, 14, 0, 4), O.MMSE),
                 (synth.Shape(13, 5, 512, 301, 6, 0, 2), O.ZF),            # ragged last group
                 (synth.Shape(8, 1, 512, 64, 3, 0, 6), O.MMSE),            # one user
                 (synth.Shape(64, 15, 2048, 1200, 14, 0, 4), O.ZF)]


@pytest.mark.parametrize("sh,det", PRECODE_CASES)
def test_precode_vs_oracle_and_zf_loopback(rx, sh, det):
    """X against the oracle's precoder on the GPU's own yf (relative RMS over
    subcarriers with kappa_2(A) <= 1e3), identical flags (a zero pilot makes a
    non-finite estimate), zeros where flagged, and for ZF H^H X = S."""
    frs = [synth.make_frame(4, f, shape=sh) for f in range(2)]
    x = dev(np.stack([f.x for f in frs]))
    p = dev(np.stack([f.pilots for f in frs]))
    p[1, 7] = 0
    fr = rx.Frame.of(sh, det, 1.0)
    yf = rx.fft(fr, x)
    rng = np.random.default_rng([23, sh.M, sh.n_sc])
    bits = rng.integers(0, 2, (2, sh.K, sh.n_data, sh.n_sc, sh.qam_bits)).astype(np.uint8)
    s = rx.modulate(fr, dev(bits))
    xf, fl = rx.precode(fr, yf, p, s)
    torch.cuda.synchronize()
    yh, ph, sh_, xh, flh = host(yf), host(p), host(s), host(xf), host(fl)
    for f in range(2):
        H = O.csi_stage(yh[f][:, 0, :], ph[f], sh.K)
        ref = O.precode_stage(H, sh_[f], 1.0, det)
        A = O.regularised_gram(np.moveaxis(np.where(np.isfinite(H), H, 0), -1, 0), 1.0, det)
        ev = np.linalg.eigvalsh(A)
        with np.errstate(divide="ignore", invalid="ignore"):
            kap = ev[:, -1] / ev[:, 0]
        good = (kap <= 1e3) & (ref["flags"] == 0)
        assert np.array_equal(flh[f], ref["flags"])
        assert not xh[f][..., ref["flags"] != 0].any()
        e = rel_rms(xh[f][..., good], ref["x"][..., good])
        msg = ["frame", f, "rel_rms", e, "subcarriers", int(good.sum()), "flagged", int((ref["flags"] != 0).sum())]
        assert e < 1e-4
        if det == O.ZF:
            back = np.einsum("mki,mdi->kdi", np.conj(H[..., good]), xh[f][..., good].astype(np.complex128))
            el = rel_rms(back, sh_[f][..., good])
            msg += ["loopback rel_rms", el]
            assert el < 1e-4
        say("precode", sh, "ZF" if det == O.ZF else "MMSE", *msg)


def test_precode_workspace_only_for_sixteen_users(rx):
    """16 users use the factor records in the workspace; fewer need none."""
    for K, need in ((16, True), (8, False), (1, False)):
        sh = synth.Shape(32, K, 512, 300, 6, 0, 2)
        fr = rx.Frame.of(sh, rx.ZF, 1.0)
        assert (rx.workspace_bytes(fr, 2, rx.WS_PRECODE, "fp32") > 0) == need


def test_downlink_bench_launch_sampled_frames(rx):
    """The 100-frame 64x16 downlink exactly as the benchmark launches it (one
    modulate, one precode and one inverse-transform call over all frames);
    sampled frames checked against the oracle."""
    sh = synth.config_shape(2)
    res = synth.draw_inputs(2, range(100), workers=8)
    x = dev(np.stack([r[0] for r in res]))
    p = dev(np.stack([r[1] for r in res]))
    fr = rx.Frame.of(sh, rx.ZF, 1.0)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    bits = torch.randint(0, 2, (100, sh.K, sh.n_data, sh.n_sc, sh.qam_bits), generator=g, device="cuda",
                         dtype=torch.uint8)
    yf = rx.fft(fr, x)
    del x
    s = rx.modulate(fr, bits)
    xf, fl = rx.precode(fr, yf, p, s)
    xt = rx.ifft(fr, xf)
    torch.cuda.synchronize()
    for f in (0, 57, 99):
        bh, sh_, yh, ph = host(bits[f]), host(s[f]), host(yf[f]), host(p[f])
        assert np.max(np.abs(sh_ - O.modulate_stage(bh, sh.qam_bits))) < 4 * 2.0 ** -23
        H = O.csi_stage(yh[:, 0, :], ph, sh.K)
        ref = O.precode_stage(H, sh_, 1.0, O.ZF)
        assert np.array_equal(host(fl[f]), ref["flags"])
        e = rel_rms(host(xf[f]), ref["x"])
        t = O.ifft_stage(host(xf[f]), sh.n_fft, sh.n_sc, sh.cp_len)
        e2 = rel_rms(host(xt[f]), t)
        say("100-frame downlink, frame", f, "precode rel_rms", e, "ifft rel_rms", e2)
        assert e < 1e-4 and e2 < 2e-6


@pytest.mark.parametrize("det", [0, 1])
def test_precode_reuses_the_uplink_factors(rx, det):
    """After the fused uplink call (csi_detect_demod, and csi_detect) on the
    same frames, precoding with its workspace's factor records gives exactly
    what refactoring gives."""
    sh = synth.Shape(64, 16, 2048, 1200, 14, 0, 4)
    frs = [synth.make_frame(4, 20 + f, shape=sh) for f in range(3)]
    x = dev(np.stack([f.x for f in frs]))
    p = dev(np.stack([f.pilots for f in frs]))
    p[2, 30] = 0
    fr = rx.Frame.of(sh, det, 1.0)
    yf = rx.fft(fr, x)
    rng = np.random.default_rng([24, det])
    s = rx.modulate(fr, dev(rng.integers(0, 2, (3, sh.K, sh.n_data, sh.n_sc, sh.qam_bits)).astype(np.uint8)))
    ref_x, ref_f = rx.precode(fr, yf, p, s)
    for kind in (rx.WS_CSI_DETECT_DEMOD, rx.WS_CSI_DETECT):
        ws = torch.empty((rx.workspace_bytes(fr, 3, kind, "fp32"),), dtype=torch.uint8, device="cuda")
        if kind == rx.WS_CSI_DETECT_DEMOD:
            rx.csi_detect_demod(fr, yf, p, ws=ws)
        else:
            rx.csi_detect(fr, yf, p, ws=ws)
        xf, fl = rx.precode(fr, yf, p, s, ws=ws, reuse_factors=True)
        torch.cuda.synchronize()
        assert torch.equal(xf, ref_x) and torch.equal(fl, ref_f), kind


def test_empty_calls_are_no_ops(rx):
    """Zero frames or rows: every downlink and 16-bit call returns OK and
    touches nothing."""
    import ctypes
    lib = rx.load()
    for K in (16, 4):
        sh = synth.Shape(16, K, 512, 300, 6, 0, 2)
        fr = rx.Frame.of(sh, rx.ZF, 1.0)
        c = ctypes.byref(fr.c())
        sentinel = torch.full((64,), 7, dtype=torch.uint8, device="cuda")
        p = ctypes.c_void_p(sentinel.data_ptr())
        assert lib.rxphy_modulate(c, 0, None, None, None) == 0
        assert lib.rxphy_precode(c, 0, None, None, None, None, None, None, 0, 0, None) == 0
        assert lib.rxphy_ifft(c, 0, None, None, None) == 0
        assert lib.rxphy_ifft_sc16(c, 0, None, 1.0, None, None) == 0
        assert lib.rxphy_fft_sc16(c, 0, None, 1.0, None, None) == 0
        assert lib.rxphy_ifft(c, -1, p, p, None) == 1
        torch.cuda.synchronize()
        assert (sentinel == 7).all()


@pytest.mark.parametrize("sh,det", [(synth.Shape(64, 16, 2048, 1200, 14, 0, 4), 0),
                                    (synth.Shape(21, 16, 512, 500, 17, 0, 2), 1),
                                    (synth.Shape(64, 16, 4096, 3276, 5, 0, 6), 0),
                                    (synth.Shape(32, 8, 1024, 600, 14, 0, 6), 1),
                                    (synth.Shape(13, 5, 512, 301, 6, 0, 2), 0),
                                    (synth.Shape(8, 1, 512, 64, 3, 0, 4), 1)])
def test_modulate_precode_equals_the_two_calls(rx, sh, det):
    """The fused call maps each point from its bit bytes where the precoder
    reads it: xf and flags equal modulate + precode bit for bit (also with
    the uplink's factor records reused for 16 users)."""
    frs = [synth.make_frame(4, 30 + f, shape=sh) for f in range(2)]
    x = dev(np.stack([f.x for f in frs]))
    p = dev(np.stack([f.pilots for f in frs]))
    p[1, 5] = 0
    fr = rx.Frame.of(sh, det, 1.0)
    yf = rx.fft(fr, x)
    rng = np.random.default_rng([25, sh.K, sh.qam_bits])
    bits = dev((rng.integers(0, 2, (2, sh.K, sh.n_data, sh.n_sc, sh.qam_bits)) * rng.integers(1, 4, 1)[0]).astype(np.uint8))
    ref_x, ref_f = rx.precode(fr, yf, p, rx.modulate(fr, bits))
    xf, fl = rx.modulate_precode(fr, yf, p, bits)
    torch.cuda.synchronize()
    assert torch.equal(xf, ref_x) and torch.equal(fl, ref_f)
    if sh.K == 16:
        ws = torch.empty((rx.workspace_bytes(fr, 2, rx.WS_CSI_DETECT_DEMOD, "fp32"),), dtype=torch.uint8, device="cuda")
        rx.csi_detect_demod(fr, yf, p, ws=ws)
        xr, flr = rx.modulate_precode(fr, yf, p, bits, ws=ws, reuse_factors=True)
        torch.cuda.synchronize()
        assert torch.equal(xr, ref_x) and torch.equal(flr, ref_f)
