"""GPU parity: every stage of librxphy against the FP64 oracle on the same
seeded inputs (per stage, with the GPU's own upstream output as the common
input, and for the whole chain from the complex64 samples)."""
import math

import numpy as np
import pytest

import oracle as O
import synth
from parity_util import evm_rel, hard_bits_outside_guard, llr_rel, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-parity]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def frames_to_device(frs):
    x = dev(np.stack([f.x for f in frs]))
    p = dev(np.stack([f.pilots for f in frs]))
    return x, p


# ------------------------------------------------------------------ stage: fft
@pytest.mark.parametrize("N,n_sc,cp", [(512, 300, 0), (1024, 601, 7), (2048, 1200, 0),
                                       (4096, 3276, 0), (4096, 4096, 288), (512, 17, 36)])
def test_fft_stage(rx, N, n_sc, cp):
    say("fft", N, n_sc, cp)
    rng = np.random.default_rng(N + n_sc)
    M, S, F = 3, 4, 2
    x = (rng.standard_normal((F, M, S, cp + N)) + 1j * rng.standard_normal((F, M, S, cp + N))).astype(np.complex64)
    fr = rx.Frame(M, 1, N, n_sc, S, cp, 2)
    yf = host(rx.fft(fr, dev(x)))
    torch.cuda.synchronize()
    ref = O.fft_stage(x, N, n_sc, cp)
    e = rel_rms(yf, ref)
    say("  rel rms", e, "max abs", float(np.max(np.abs(yf - ref))))
    assert e < 2e-6
    assert np.max(np.abs(yf - ref)) < 1e-5 * np.max(np.abs(ref))


def test_fft_impulse_and_tone(rx):
    N, n_sc = 2048, 1200
    x = np.zeros((1, 1, 2, N), np.complex64)
    x[0, 0, 0, 5] = 1.0
    i0 = 77
    k0 = (i0 - n_sc // 2) % N
    x[0, 0, 1] = np.exp(2j * np.pi * k0 * np.arange(N) / N).astype(np.complex64)
    yf = host(rx.fft(rx.Frame(1, 1, N, n_sc, 2, 0, 2), dev(x)))
    k = (np.arange(n_sc) - n_sc // 2) % N
    np.testing.assert_allclose(yf[0, 0, 0], np.exp(-2j * np.pi * k * 5 / N), atol=2e-6)
    ref = np.zeros(n_sc, complex)
    ref[i0] = N
    np.testing.assert_allclose(yf[0, 0, 1], ref, atol=2e-3)


# ------------------------------------------------------------------ stage: csi
@pytest.mark.parametrize("M,K,n_sc", [(8, 2, 300), (64, 16, 1200), (12, 5, 301), (4, 1, 40), (16, 16, 99)])
def test_csi_stage(rx, M, K, n_sc):
    say("csi", M, K, n_sc)
    rng = np.random.default_rng(M * K + n_sc)
    F, S = 2, 3
    yf = (rng.standard_normal((F, M, S, n_sc)) + 1j * rng.standard_normal((F, M, S, n_sc))).astype(np.complex64)
    p = synth.qam_map(rng.integers(0, 2, (F, n_sc, 2)), 2).astype(np.complex64) * np.float32(1.3)
    fr = rx.Frame(M, K, 512 if n_sc <= 512 else 2048, n_sc, S, 0, 2)
    h = host(rx.csi(fr, dev(yf), dev(p)))
    for f in range(F):
        ref = O.csi_stage(yf[f, :, 0, :], p[f], K)
        assert rel_rms(h[f], ref) < 1e-6


# --------------------------------------------------------------- stage: detect
DETECT_CASES = [
    # M, K, n_sc, n_sym, detector, snr range
    (8, 2, 300, 14, O.ZF, (20, 20)),
    (64, 16, 1200, 14, O.ZF, (10, 30)),
    (64, 16, 1200, 14, O.MMSE, (10, 30)),
    (12, 5, 77, 14, O.MMSE, (0, 15)),      # M not a multiple of 8, ragged tile
    (16, 16, 50, 14, O.ZF, (25, 25)),      # K = M
    (8, 1, 33, 5, O.ZF, (5, 5)),           # one user, short frame
    (64, 16, 41, 17, O.MMSE, (10, 30)),    # 16 data symbols
    (3, 3, 20, 2, O.MMSE, (10, 10)),       # tiny M, one data symbol
]


@pytest.mark.parametrize("M,K,n_sc,S,det,snr", DETECT_CASES)
def test_detect_stage(rx, M, K, n_sc, S, det, snr):
    say("detect", M, K, n_sc, S, det, snr)
    N = 512 if n_sc <= 512 else 2048
    sh = synth.Shape(M, K, N, n_sc, S, 0, 4)
    frs = [synth.make_frame(11, f, shape=sh, snr=snr) for f in range(2)]
    x, p = frames_to_device(frs)
    fr = rx.Frame.of(sh, det, 1.0)
    yf = rx.fft(fr, x)
    h = rx.csi(fr, yf, p)
    xt, nu, fl = rx.detect(fr, h, yf)
    torch.cuda.synchronize()
    yf, h, xt, nu, fl = host(yf), host(h), host(xt), host(nu), host(fl)
    for f in range(2):
        ref = O.detect_stage(h[f], yf[f, :, 1:, :], 1.0, det, want_kappa=True)
        good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
        assert np.array_equal(fl[f], ref["flags"])
        e = evm_rel(xt[f], ref["xt"], good)
        en = rel_rms(nu[f][:, good], ref["nu"][:, good])
        say("  frame", f, "evm_rel", e, "nu_rel", en, "kappa max", float(ref["kappa"].max()))
        assert e < 1e-4
        assert en < 1e-4


def test_detect_flags_and_erasures(rx):
    M, K, n_sc, S = 8, 3, 40, 4
    rng = np.random.default_rng(3)
    h = (rng.standard_normal((1, M, K, n_sc)) + 1j * rng.standard_normal((1, M, K, n_sc))).astype(np.complex64)
    yf = (rng.standard_normal((1, M, S, n_sc)) + 1j * rng.standard_normal((1, M, S, n_sc))).astype(np.complex64)
    h[0, :, 1, 5] = 0          # zero column -> breakdown (ZF) / mu = 0 (MMSE)
    h[0, 2, 0, 9] = np.nan     # non-finite channel
    yf[0, 4, 2, 20] = np.inf   # non-finite data
    for det in (O.ZF, O.MMSE):
        fr = rx.Frame(M, K, 512, n_sc, S, 0, 2, det, 1.0)
        xt, nu, fl = (host(t) for t in rx.detect(fr, dev(h), dev(yf)))
        ref = O.detect_stage(h[0], yf[0, :, 1:, :], 1.0, det)
        assert np.array_equal(fl[0], ref["flags"]), (fl[0], ref["flags"])
        bad = ref["flags"] != 0
        assert np.all(xt[0][..., bad] == 0) and np.all(np.isinf(nu[0][:, bad]))
        llr = host(rx.demod(fr, dev(xt), dev(nu)))
        assert np.all(llr[0][:, :, bad] == 0)


@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_detect_shared_factor_tiles(rx, det):
    """Tiles whose 16 subcarriers carry one channel matrix (a pilot group of
    K = 16) factor A once; tiles broken by a perturbed or non-finite entry, and
    groups that break down, must give the per-subcarrier results."""
    M, K, n_sc, S = 32, 16, 200, 6          # 12 groups, the last one 24 subcarriers wide
    rng = np.random.default_rng(17 + det)
    G = n_sc // K
    hg = (rng.standard_normal((M, K, G)) + 1j * rng.standard_normal((M, K, G))) * 0.7
    gidx = np.minimum(np.arange(n_sc) // K, G - 1)
    h = hg[:, :, gidx][None].astype(np.complex64)
    yf = (rng.standard_normal((1, M, S, n_sc)) + 1j * rng.standard_normal((1, M, S, n_sc))).astype(np.complex64) * 3
    h[0, 5, 3, 37] *= np.float32(1 + 1e-3)  # tile 2 no longer uniform
    h[0, 1, 2, 70] = np.nan                 # tile 4: non-finite channel on one subcarrier
    h[0, :, 9, 96:112] = 0                  # group 6: a zero user column -> breakdown (ZF) / mu = 0 (MMSE)
    yf[0, 3, 2, 150] = np.inf               # non-finite data on one subcarrier of a uniform tile
    fr = rx.Frame(M, K, 512, n_sc, S, 0, 2, det, 1.0)
    xt, nu, fl = (host(t) for t in rx.detect(fr, dev(h), dev(yf)))
    ref = O.detect_stage(h[0], yf[0, :, 1:, :], 1.0, det, want_kappa=True)
    assert np.array_equal(fl[0], ref["flags"]), (np.nonzero(fl[0] != ref["flags"]), fl[0], ref["flags"])
    good = (ref["flags"] == 0) & (ref["kappa"] <= 1e3)
    e = evm_rel(xt[0], ref["xt"], good)
    en = rel_rms(nu[0][:, good], ref["nu"][:, good])
    say("shared-factor tiles", det, "evm_rel", e, "nu_rel", en, "flagged", int(np.sum(~good)))
    assert e < 1e-4 and en < 1e-4
    bad = ref["flags"] != 0
    assert np.all(xt[0][..., bad] == 0) and np.all(np.isinf(nu[0][:, bad]))


# ---------------------------------------------------------------- stage: demod
@pytest.mark.parametrize("q", [2, 4, 6])
def test_demod_stage(rx, q):
    say("demod", q)
    rng = np.random.default_rng(q)
    F, K, D, n_sc = 2, 3, 5, 333
    xt = (rng.standard_normal((F, K, D, n_sc)) + 1j * rng.standard_normal((F, K, D, n_sc))).astype(np.complex64)
    nu = rng.uniform(0.01, 3.0, (F, K, n_sc)).astype(np.float32)
    nu[0, 1, 7] = np.inf
    fr = rx.Frame(8, K, 512, n_sc, D + 1, 0, q)
    llr = host(rx.demod(fr, dev(xt), dev(nu)))
    # Each LLR within the FP32 forward-error bound of its definition (a
    # difference of two squared distances along one axis, divided by nu):
    # every operand is at most |x| + l_max, so any evaluation order in FP32
    # errs by at most a few units of 2^-24 (|x| + l_max)^2 / nu, plus the
    # rounding of the result; and the relative metric below 1e-4, a tenth of
    # the stated LLR target.  The metric cannot be held to 1e-5 here: the
    # inputs are Gaussian, wider than the constellation, with nu down to
    # 0.01, so an LLR near zero at the smallest nu carries an absolute error
    # of that bound, up to 1.4e-5 of the metric's floor (0.01 RMS) for 64-QAM,
    # while staying within a quarter of its own FP32 bound.
    lmax = {2: 1 / math.sqrt(2), 4: 3 / math.sqrt(10), 6: 7 / math.sqrt(42)}[q]
    u = 2.0 ** -24
    for f in range(F):
        ref = O.demod_stage(xt[f], nu[f], q)
        e = llr_rel(llr[f], ref)
        ax = np.stack([(xt[f].real if j % 2 == 0 else xt[f].imag) for j in range(q)], axis=-1).astype(np.float64)
        bound = 8 * u * (np.abs(ax) + lmax) ** 2 / nu[f][:, None, :, None] + 2 * u * np.abs(ref)
        fin = ~np.broadcast_to(np.isinf(nu[f])[:, None, :, None], ref.shape)
        worst = float(np.max(np.abs(llr[f] - ref)[fin] / bound[fin]))
        say("  llr_rel", e, "max error / FP32 bound", worst)
        assert e < 1e-4
        assert worst <= 1.0
        assert np.all(llr[f][~fin] == 0)            # erased points
        mism, band = hard_bits_outside_guard(llr[f], ref)
        assert mism == 0


@pytest.mark.parametrize("q", [2, 4, 6])
def test_demod_midpoints_and_large_values(rx, q):
    """The nearest levels are found in closed form, not by a search: the LLRs
    at and next to every decision midpoint (even multiples of the level unit)
    and at large |x_tilde| still follow the definition within the FP32 bound
    of test_demod_stage, and at huge |x_tilde|, where squared distances would
    overflow FP32, they stay finite, carry the sign of the nearest outer
    level and double when x_tilde doubles (the max-log LLR is affine there)."""
    c = {2: 1 / math.sqrt(2), 4: 1 / math.sqrt(10), 6: 1 / math.sqrt(42)}[q]
    lmax = {2: 1, 4: 3, 6: 7}[q] * c
    mids = np.array([k * c for k in range(-8, 9, 2)], dtype=np.float32)
    near = np.concatenate([mids, np.nextafter(mids, np.float32(np.inf)), np.nextafter(mids, np.float32(-np.inf))])
    big = np.array([10.0, -37.5, 1e3, -1e3, 2.5e5, -1e6], dtype=np.float32)
    axis = np.concatenate([near, big]).astype(np.float32)
    n_ax = axis.size
    re, im = np.meshgrid(axis, axis[::-1], indexing="ij")
    n_sc = n_ax * n_ax
    xt = (re + 1j * im).astype(np.complex64).reshape(1, 1, 1, n_sc)
    nu = np.full((1, 1, n_sc), 0.37, dtype=np.float32)
    fr = rx.Frame(8, 1, 4096, n_sc, 2, 0, q)
    llr = host(rx.demod(fr, dev(xt), dev(nu)))[0]
    ref = O.demod_stage(xt[0], nu[0], q)
    u = 2.0 ** -24
    ax = np.stack([(xt[0].real if j % 2 == 0 else xt[0].imag) for j in range(q)], axis=-1).astype(np.float64)
    # plus the oracle's own rounding: it differences complex squared
    # distances in FP64, in which the other axis' term (up to (1e6)^2 here)
    # cancels only to a few units of 2^-53 of its size
    both = (np.abs(xt[0].real) + np.abs(xt[0].imag) + 2 * lmax)[..., None].astype(np.float64)
    bound = 8 * u * (np.abs(ax) + lmax) ** 2 / 0.37 + 2 * u * np.abs(ref) + 8 * 2.0 ** -53 * both ** 2 / 0.37
    worst = float(np.max(np.abs(llr - ref) / bound))
    say("demod midpoints / large", q, "max error / FP32 bound", worst)
    assert worst <= 1.0

    huge = np.array([1e15, -3e20, 7e25, -1e30], dtype=np.float32)
    hc = (huge + 1j * huge[::-1]).astype(np.complex64)
    x2 = np.concatenate([hc, 2 * hc]).astype(np.complex64)
    xt2 = x2.reshape(1, 1, 1, -1)
    nu2 = np.full((1, 1, x2.size), 0.37, dtype=np.float32)
    fr2 = rx.Frame(8, 1, 512, x2.size, 2, 0, q)
    l2 = host(rx.demod(fr2, dev(xt2), dev(nu2)))[0, 0, 0]           # [n, q]
    assert np.all(np.isfinite(l2))
    n = huge.size
    assert np.array_equal(l2[n:], 2 * l2[:n])                        # affine with no offset at this scale
    sgn = np.sign(np.stack([x2.real, x2.imag], axis=-1))             # in-phase, quadrature coordinate
    assert np.array_equal(np.sign(l2[:, 0]), sgn[:, 0])             # sign bits: positive axis -> b = 0
    assert np.array_equal(np.sign(l2[:, 1]), sgn[:, 1])
    if q > 2:                                                        # inner bits of the outer level are ones
        assert np.all(l2[:, 2:] < 0)


@pytest.mark.parametrize("q", [2, 4, 6])
def test_demod_non_finite_coordinates(rx, q):
    """A non-finite coordinate of x_tilde with a finite nu gives non-finite LLRs
    for the bits of that axis only (the other axis' bits equal those of the
    same point with that coordinate finite); an erased stream (nu = inf)
    gives zeros whatever x_tilde holds."""
    vals = np.array([np.nan, np.inf, -np.inf], dtype=np.float32)
    fin = np.float32(0.3)
    xt = np.empty(9, dtype=np.complex64)                 # parts set one by one (1j * inf is nan + inf j)
    xt.real = np.concatenate([vals, np.full(3, fin), vals])
    xt.imag = np.concatenate([np.full(3, fin), vals, vals])
    ref_pt = np.full(xt.shape, fin + 1j * fin, dtype=np.complex64)
    n = xt.size
    nu = np.full((1, 1, 2 * n), 0.5, dtype=np.float32)
    nu[0, 0, -1] = np.inf
    x_all = np.concatenate([xt, ref_pt]).reshape(1, 1, 1, 2 * n)
    x_all[0, 0, 0, -1] = np.complex64(np.nan + 1j * np.nan)        # erased stream with a NaN point
    fr = rx.Frame(8, 1, 512, 2 * n, 2, 0, q)
    llr = host(rx.demod(fr, dev(x_all), dev(nu)))[0, 0, 0]        # [2n, q]
    bad, good = llr[:n], llr[n:]
    re_bits, im_bits = np.arange(0, q, 2), np.arange(1, q, 2)
    assert np.all(~np.isfinite(bad[:3][:, re_bits])) and np.array_equal(bad[:3][:, im_bits], good[:3][:, im_bits])
    assert np.all(~np.isfinite(bad[3:6][:, im_bits])) and np.array_equal(bad[3:6][:, re_bits], good[3:6][:, re_bits])
    assert np.all(~np.isfinite(bad[6:9]))
    assert np.all(llr[-1] == 0)


# ------------------------------------------------------------------ full chain
CHAIN_CASES = [(1, O.ZF, 1), (2, O.ZF, 2), (2, O.MMSE, 2), (3, O.ZF, 1)]


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("cfg,det,nfr", CHAIN_CASES)
def test_chain_vs_oracle(rx, cfg, det, nfr, fused):
    say("chain", cfg, det, nfr, "fused" if fused else "staged")
    frs = synth.make_frames(cfg, nfr)
    sh = frs[0].shape
    x, p = frames_to_device(frs)
    fr = rx.Frame.of(sh, det, 1.0)
    out = {k: host(v) for k, v in rx.forward(fr, x, p, fused=fused).items()}
    for f, fo in enumerate(frs):
        ref = O.forward(fo.x, fo.pilots, sh, 1.0, det, want_kappa=True)
        good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
        e = evm_rel(out["xt"][f], ref["xt"], good)
        l = llr_rel(out["llr"][f], ref["llr"])
        mism, band = hard_bits_outside_guard(out["llr"][f], ref["llr"])
        ber = float(np.mean(O.hard_bits(out["llr"][f]) != fo.bits))
        say("  frame", f, "evm_rel", e, "llr_rel", l, "hard mismatches", mism, "in band", band, "BER", ber)
        assert np.array_equal(out["flags"][f], ref["flags"])
        assert e < 1e-4
        assert l < 1e-3
        assert mism == 0


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_chain_at_maximum_shape(rx, det, fused):
    """M 64, K 16, N 4096 with every bin used, 17 symbols, 64-QAM."""
    sh = synth.Shape(64, 16, 4096, 4096, 17, 0, 6)
    fo = synth.make_frame(3, 0, shape=sh, snr=(20, 30))
    x, p = frames_to_device([fo])
    fr = rx.Frame.of(sh, det, 1.0)
    out = {k: host(v) for k, v in rx.forward(fr, x, p, fused=fused).items()}
    ref = O.forward(fo.x, fo.pilots, sh, 1.0, det, want_kappa=True)
    good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
    e = evm_rel(out["xt"][0], ref["xt"], good)
    l = llr_rel(out["llr"][0], ref["llr"])
    mism, band = hard_bits_outside_guard(out["llr"][0], ref["llr"])
    say("max shape", det, "evm_rel", e, "llr_rel", l, "hard mismatches", mism, "in band", band)
    assert np.array_equal(out["flags"][0], ref["flags"])
    assert e < 1e-4 and l < 1e-3 and mism == 0


def test_headline_launch_sampled_frames(rx):
    """The 100-frame 64x16 batch exactly as the benchmark launches it (one call
    per stage over all frames); sampled frames checked against the oracle."""
    sh = synth.config_shape(2)
    res = synth.draw_inputs(2, range(100), workers=8)
    x = dev(np.stack([r[0] for r in res]))
    p = dev(np.stack([r[1] for r in res]))
    fr = rx.Frame.of(sh, O.ZF, 1.0)
    out = rx.forward(fr, x, p, fused=True)          # the benchmark's path
    staged = rx.forward(fr, x, p)
    torch.cuda.synchronize()
    assert_fused_matches(out["xt"], out["nu"], out["flags"], staged["xt"], staged["nu"], staged["flags"])
    for f in (0, 41, 99):
        ref = O.forward(res[f][0], res[f][1], sh, 1.0, O.ZF, want_kappa=True)
        good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
        e = evm_rel(host(out["xt"][f]), ref["xt"], good)
        llr = host(out["llr"][f])
        l = llr_rel(llr, ref["llr"])
        mism, band = hard_bits_outside_guard(llr, ref["llr"])
        say("100-frame launch, frame", f, "evm_rel", e, "llr_rel", l, "hard mismatches", mism)
        assert np.array_equal(host(out["flags"][f]), ref["flags"])
        assert e < 1e-4 and l < 1e-3 and mism == 0


FUSED_CASES = [(synth.Shape(64, 16, 2048, 1200, 14, 0, 4), O.ZF, "fp32"),
               (synth.Shape(64, 16, 2048, 1200, 14, 0, 4), O.MMSE, "bf16"),
               (synth.Shape(32, 16, 1024, 601, 9, 16, 6), O.MMSE, "fp32"),
               (synth.Shape(16, 5, 1024, 777, 14, 0, 2), O.ZF, "fp16"),
               (synth.Shape(8, 1, 512, 300, 14, 0, 2), O.MMSE, "fp32"),
               (synth.Shape(64, 12, 4096, 3276, 17, 0, 6), O.ZF, "fp32"),
               # 16 users: one pilot group per tile (the group kernel): antennas
               # not a multiple of 4, 16 and 1 data symbols, square M = K, ragged ends
               (synth.Shape(21, 16, 512, 500, 17, 0, 4), O.MMSE, "fp32"),
               (synth.Shape(64, 16, 1024, 1000, 2, 0, 2), O.MMSE, "fp32"),
               (synth.Shape(16, 16, 512, 200, 6, 8, 4), O.ZF, "fp32"),
               (synth.Shape(64, 16, 4096, 3276, 17, 0, 6), O.MMSE, "fp32")]


def assert_fused_matches(xt_f, nu_f, fl_f, xt_s, nu_s, fl_s, exact=False):
    """Fused vs staged outputs.  Flags and noise variances come from the same
    factorisation and are identical, and so are the erasures; with exact=False
    (16 users in FP32, where the fused path applies the explicit inverse on
    MFMA instead of the two triangular solves) x_tilde is checked against the
    oracle by the caller instead of bit for bit."""
    assert torch.equal(fl_f, fl_s)
    assert torch.equal(nu_f, nu_s)
    a, b = torch.view_as_real(xt_f), torch.view_as_real(xt_s)
    if exact:
        assert torch.equal(a, b)
        return
    assert torch.equal(a == 0, b == 0)
    rel = float((a.double() - b.double()).pow(2).sum().sqrt() / b.double().pow(2).sum().sqrt())
    say("  fused vs staged: relative RMS difference", rel)


@pytest.mark.parametrize("sh,det,prec", FUSED_CASES)
def test_fused_csi_detect_equals_two_calls(rx, sh, det, prec):
    """rxphy_csi_detect against rxphy_csi followed by rxphy_detect (every K
    padding, ragged tiles, both detectors, the refined forms, a zero pilot,
    non-finite data values, and a threshold that refines): bit-identical,
    except x_tilde of the 16-user FP32 path (see assert_fused_matches)."""
    frs = [synth.make_frame(4, f, shape=sh) for f in range(2)]
    x, p = frames_to_device(frs)
    p[1, 7] = 0                                     # zero pilot: non-finite estimates, flagged
    fr = rx.Frame.of(sh, det, 1.0)
    yf = rx.fft(fr, x)
    yf[0, 0, 1, 17] = float("nan")                  # non-finite data values: flagged subcarriers
    yf[1, sh.M - 1, sh.n_sym - 1, 40] = float("inf")
    thr = 20.0 if prec != "fp32" else 1e3           # low threshold: some subcarriers refined
    a = rx.detect(fr, rx.csi(fr, yf, p), yf, prec, thr)
    b = rx.csi_detect(fr, yf, p, prec, thr)
    torch.cuda.synchronize()
    refined = int((a[2] & rx.FLAG_REFINED).ne(0).sum().item())
    say("fused", sh, det, prec, "refined", refined, "flagged", int(a[2].ne(0).sum().item()))
    exact = not (sh.K == 16 and prec == "fp32")
    assert_fused_matches(b[0], b[1], b[2], a[0], a[1], a[2], exact=exact)
    if not exact:
        yh, ph, xf = host(yf), host(p), host(b[0])
        for f in range(len(frs)):
            H = O.csi_stage(yh[f][:, 0, :], ph[f], sh.K)
            ref = O.detect_stage(H, yh[f][:, 1:, :], 1.0, det, want_kappa=True)
            good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
            e = evm_rel(xf[f], ref["xt"], good)
            say("  fused frame", f, "evm_rel vs oracle", e, "subcarriers", int(good.sum()))
            assert e < 1e-4


@pytest.mark.parametrize("sh,det,prec", FUSED_CASES)
def test_fused_csi_detect_demod_equals_stages(rx, sh, det, prec):
    """rxphy_csi_detect_demod gives the llr, nu and flags of rxphy_csi_detect
    followed by rxphy_demod bit for bit (x_tilde too when asked for), with and
    without x_tilde written, on the same zero pilot and non-finite values."""
    frs = [synth.make_frame(4, f, shape=sh) for f in range(2)]
    x, p = frames_to_device(frs)
    p[1, 7] = 0
    fr = rx.Frame.of(sh, det, 1.0)
    yf = rx.fft(fr, x)
    yf[0, 0, 1, 17] = float("nan")
    yf[1, sh.M - 1, sh.n_sym - 1, 40] = float("inf")
    thr = 20.0 if prec != "fp32" else 1e3
    xt, nu, fl = rx.csi_detect(fr, yf, p, prec, thr)
    llr = rx.demod(fr, xt, nu)
    for want_xt in (False, True):
        l2, nu2, fl2, xt2 = rx.csi_detect_demod(fr, yf, p, prec, thr, want_xt=want_xt)
        torch.cuda.synchronize()
        assert torch.equal(l2, llr) and torch.equal(nu2, nu) and torch.equal(fl2, fl)
        if want_xt:
            assert torch.equal(torch.view_as_real(xt2), torch.view_as_real(xt))
        else:
            assert xt2 is None
    say("fused demod", sh, det, prec, "erased", int(fl.ne(0).sum().item()))


def test_deterministic(rx):
    frs = synth.make_frames(2, 1)
    x, p = frames_to_device(frs)
    fr = rx.Frame.of(frs[0].shape, O.MMSE, 1.0)
    a = rx.forward(fr, x, p)
    b = rx.forward(fr, x, p)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_zero_frames_and_shape_errors(rx):
    fr = rx.Frame(8, 2, 512, 300, 14, 0, 2)
    x = torch.empty((0, 8, 14, 512), dtype=torch.complex64, device="cuda")
    assert rx.fft(fr, x).shape == (0, 8, 14, 300)
    with pytest.raises(rx.RxphyError):
        rx.fft(fr, torch.empty((1, 8, 14, 500), dtype=torch.complex64, device="cuda"))
