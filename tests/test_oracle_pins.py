"""Pins of the FP64 oracle against things other than itself: naive DFTs,
Parseval, closed forms, library factorisations, brute-force ML, adjoint
identities and finite differences.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def crandn(rng, shape, scale=1.0):
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


# ----------------------------------------------------------------------- framing
def test_paper_fft_framing_numbers():
    g = json.load(open(os.path.join(GOLDEN, "paper_framing.json")))
    dt, df, rate32 = synth.fft_framing(g["n_fft"], g["fs_hz"], 64)
    _, _, rate16 = synth.fft_framing(g["n_fft"], g["fs_hz"], 32)
    assert dt * 1e6 == pytest.approx(g["dt_us"], rel=1e-12)
    assert df / 1e3 == pytest.approx(g["df_khz"], abs=0.1)
    assert rate32 / 1e9 == pytest.approx(g["fft_rate_gbps_32bit_iq"], rel=1e-12)
    assert rate16 / 1e9 == pytest.approx(g["raw_rate_gbps_16bit_iq"], rel=1e-12)
    assert g["tf_window_T"] * dt * 1e3 == pytest.approx(g["tf_window_ms"], rel=1e-12)


# --------------------------------------------------------------------------- fft
def naive_dft(seg):
    N = seg.shape[-1]
    n = np.arange(N)
    out = np.zeros(seg.shape, dtype=np.complex128)
    for k in range(N):
        acc = 0j
        for t in range(N):                      # the definition, term by term
            acc = acc + seg[..., t] * complex(math.cos(-2 * math.pi * k * t / N),
                                              math.sin(-2 * math.pi * k * t / N))
        out[..., k] = acc
    del n
    return out


@pytest.mark.parametrize("N,n_sc,cp", [(2, 2, 0), (4, 3, 1), (8, 5, 2), (16, 16, 0),
                                       (32, 19, 3), (64, 40, 5)])
def test_fft_stage_matches_naive_dft(N, n_sc, cp):
    rng = np.random.default_rng(N)
    x = crandn(rng, (3, 2, cp + N)).astype(np.complex64)
    got = O.fft_stage(x, N, n_sc, cp)
    full = naive_dft(x.astype(np.complex128)[..., cp:])
    for i in range(n_sc):
        k = (i - n_sc // 2) % N
        np.testing.assert_allclose(got[..., i], full[..., k], rtol=1e-12, atol=1e-12 * N)


def test_fft_stage_512_matches_naive_matrix_dft():
    N, n_sc = 512, 300
    rng = np.random.default_rng(5)
    x = crandn(rng, (2, N)).astype(np.complex64)
    n = np.arange(N)
    F = np.exp(-2j * np.pi * np.outer(n, n) / N)          # DFT matrix from its definition
    full = x.astype(np.complex128) @ F.T
    got = O.fft_stage(x, N, n_sc)
    bins = (np.arange(n_sc) - n_sc // 2) % N
    np.testing.assert_allclose(got, full[:, bins], rtol=1e-11, atol=1e-10)


def test_fft_parseval_impulse_tone_linearity():
    N = 256
    rng = np.random.default_rng(1)
    x = crandn(rng, (4, N))
    X = O.fft_stage(x, N, N)
    assert np.allclose(np.sum(np.abs(X) ** 2, -1), N * np.sum(np.abs(x) ** 2, -1), rtol=1e-12)
    # impulse at n0 -> exp(-j 2 pi k n0 / N)
    n0 = 37
    imp = np.zeros(N, complex)
    imp[n0] = 1
    Xi = O.fft_stage(imp, N, N)
    k = (np.arange(N) - N // 2) % N
    np.testing.assert_allclose(Xi, np.exp(-2j * np.pi * k * n0 / N), atol=1e-12)
    # tone at bin k0 -> N at the used subcarrier sitting on k0, zero elsewhere
    n_sc = 100
    i0 = 13
    k0 = (i0 - n_sc // 2) % N
    tone = np.exp(2j * np.pi * k0 * np.arange(N) / N)
    Xt = O.fft_stage(tone, N, n_sc)
    ref = np.zeros(n_sc, complex)
    ref[i0] = N
    np.testing.assert_allclose(Xt, ref, atol=1e-9)
    # linearity
    y = crandn(rng, (4, N))
    np.testing.assert_allclose(O.fft_stage(2 * x - 3j * y, N, 77),
                               2 * O.fft_stage(x, N, 77) - 3j * O.fft_stage(y, N, 77), atol=1e-10)


def test_fft_cp_is_skipped():
    N, cp = 64, 9
    rng = np.random.default_rng(2)
    x = crandn(rng, (N,))
    withcp = np.concatenate([rng.standard_normal(cp) * 50, x])   # garbage prefix
    np.testing.assert_allclose(O.fft_stage(withcp, N, 40, cp), O.fft_stage(x, N, 40, 0), atol=1e-12)


# --------------------------------------------------------------------------- csi
def test_csi_noiseless_recovers_block_channel():
    sh = synth.Shape(6, 3, 128, 100, 14, 4, 2)      # 100 = 33*3 + 1 trailing subcarrier
    fr = synth.make_frame(1, 0, shape=sh, n0=0.0)
    yf = O.fft_stage(fr.x, sh.n_fft, sh.n_sc, sh.cp_len)
    H = O.csi_stage(yf[:, 0, :], fr.pilots, sh.K)
    # the channel is constant over each pilot group, so LS + hold is exact
    np.testing.assert_allclose(H, fr.h, rtol=1e-5, atol=1e-5 * np.abs(fr.h).max())
    # ... and exact in FP64 when the samples are not rounded to complex64
    noise = np.zeros((sh.M, sh.n_sym, sh.n_fft))
    x64 = synth.frames.synthesize(sh, fr.h, fr.symbols, fr.pilots.astype(np.complex128), noise)
    H64 = O.csi_stage(O.fft_stage(x64, sh.n_fft, sh.n_sc, sh.cp_len)[:, 0, :],
                      fr.pilots.astype(np.complex128), sh.K)
    np.testing.assert_allclose(H64, fr.h, rtol=1e-12, atol=1e-12 * np.abs(fr.h).max())


def test_csi_noise_variance_is_n0():
    sh = synth.Shape(16, 4, 512, 400, 14, 0, 2)
    fr = synth.make_frame(7, 0, shape=sh, snr=(10.0, 10.0), n0=1.0)
    yf = O.fft_stage(fr.x, sh.n_fft, sh.n_sc)
    H = O.csi_stage(yf[:, 0, :], fr.pilots, sh.K)
    # one independent LS error per (m, pilot subcarrier of a full group)
    G = sh.n_sc // sh.K
    err = (H - fr.h)[:, :, ::sh.K][:, :, :G]
    e2 = np.abs(err) ** 2
    n = e2.size
    # |CN(0,1)|^2 is Exp(1): mean 1, std 1
    assert abs(e2.mean() - 1.0) < 5.0 / math.sqrt(n)


# ------------------------------------------------------------------------ equal
def rand_channel(rng, n_sc, M, K, scale=None):
    H = crandn(rng, (M, K, n_sc))
    if scale is not None:
        H = H * scale[None, :, None]
    return H


@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_cholesky_solve_inverse_match_numpy(det):
    rng = np.random.default_rng(3)
    M, K, D, n_sc = 12, 5, 4, 9
    H = rand_channel(rng, n_sc, M, K, scale=np.array([1, 3, 0.5, 2, 1.5]))
    Y = crandn(rng, (M, D, n_sc))
    n0 = 0.7
    Hs = np.moveaxis(H, -1, 0)
    A = O.regularised_gram(Hs, n0, det)
    L, ok = O.cholesky_lower(A)
    assert ok.all()
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(L @ np.conj(np.swapaxes(L, -1, -2)), A, rtol=1e-12, atol=1e-12)
    out = O.detect_stage(H, Y, n0, det)
    Z = np.conj(np.swapaxes(Hs, -1, -2)) @ np.moveaxis(Y, -1, 0)
    xh = np.linalg.solve(A, Z)
    np.testing.assert_allclose(np.moveaxis(out["xhat"], -1, 0), xh, rtol=1e-11, atol=1e-12)
    dinv = np.real(np.diagonal(np.linalg.inv(A), axis1=-2, axis2=-1))
    np.testing.assert_allclose(out["d"].T, dinv, rtol=1e-11)


def test_zf_noiseless_inverts_channel():
    rng = np.random.default_rng(4)
    M, K, n_sc = 16, 6, 11
    H = rand_channel(rng, n_sc, M, K)
    # W H = I: detecting Y = H column by column must give the identity
    out = O.detect_stage(H, H, 1.0, O.ZF)
    eye = np.broadcast_to(np.eye(K)[:, :, None], (K, K, n_sc))
    assert np.max(np.abs(out["xt"] - eye)) < 1e-12


def test_zf_noiseless_frame_recovers_symbols_and_bits():
    sh = synth.Shape(8, 2, 512, 300, 14, 0, 4)
    fr = synth.make_frame(1, 0, shape=sh, n0=0.0)
    o = O.forward(fr.x.astype(np.complex128), fr.pilots, sh, 1.0, O.ZF)
    # complex64 samples: symbols to ~1e-5, bits exactly
    assert np.max(np.abs(o["xt"] - fr.symbols)) < 1e-4
    assert np.array_equal(O.hard_bits(o["llr"]), fr.bits)


def test_mmse_k1_closed_forms_and_limits():
    rng = np.random.default_rng(6)
    M, D, n_sc, n0 = 7, 3, 5, 0.3
    h = crandn(rng, (M, 1, n_sc))
    y = crandn(rng, (M, D, n_sc))
    o = O.detect_stage(h, y, n0, O.MMSE)
    hh = np.sum(np.abs(h[:, 0, :]) ** 2, axis=0)                 # ||h||^2 per subcarrier
    hy = np.einsum("mi,mdi->di", np.conj(h[:, 0, :]), y)
    np.testing.assert_allclose(o["xhat"][0], hy / (hh + n0), rtol=1e-12)
    np.testing.assert_allclose(o["mu"][0], hh / (hh + n0), rtol=1e-12)
    np.testing.assert_allclose(o["xt"][0], hy / hh, rtol=1e-12)
    np.testing.assert_allclose(o["nu"][0], n0 / hh, rtol=1e-12)       # 1 / SINR
    # 0 < mu < 1, and MMSE -> ZF as N0 -> 0
    M, K = 10, 4
    H = rand_channel(rng, n_sc, M, K)
    Y = crandn(rng, (M, D, n_sc))
    o = O.detect_stage(H, Y, 0.5, O.MMSE)
    assert np.all((o["mu"] > 0) & (o["mu"] < 1))
    z = O.detect_stage(H, Y, 1.0, O.ZF)
    m = O.detect_stage(H, Y, 1e-9, O.MMSE)
    np.testing.assert_allclose(m["xt"], z["xt"], rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(m["nu"] / 1e-9, z["nu"], rtol=1e-6)


def test_breakdown_and_nonfinite_flags():
    rng = np.random.default_rng(8)
    M, K, D, n_sc = 6, 3, 2, 4
    H = rand_channel(rng, n_sc, M, K)
    Y = crandn(rng, (M, D, n_sc))
    H[:, 1, 2] = 0.0                 # zero column -> singular Gram under ZF
    Y[3, 0, 3] = np.nan              # non-finite input
    z = O.detect_stage(H, Y, 1.0, O.ZF)
    assert list(z["flags"]) == [0, 0, O.FLAG_BREAKDOWN, O.FLAG_NONFINITE]
    assert np.all(z["xt"][:, :, 2:] == 0) and np.all(np.isinf(z["nu"][:, 2:]))
    llr = O.demod_stage(z["xt"], z["nu"], 2)
    assert np.all(llr[:, :, 2:] == 0)
    m = O.detect_stage(H, Y, 1.0, O.MMSE)      # zero column under MMSE: mu = 0 -> erasure
    assert list(m["flags"]) == [0, 0, O.FLAG_BREAKDOWN, O.FLAG_NONFINITE]
    # a zero pilot makes the LS estimate non-finite
    p = np.ones(8, complex)
    p[2] = 0
    Hc = O.csi_stage(np.ones((2, 8), complex), p, 2)
    assert not np.isfinite(Hc[:, 0, 2:4]).all()


# ------------------------------------------------------------------------ demod
def test_constellations_unit_energy_gray_and_generator_agree():
    for q in (2, 4, 6):
        pts, lab = O.constellation(q)
        assert abs(np.mean(np.abs(pts) ** 2) - 1) < 1e-14
        assert len(set(np.round(pts, 12))) == 1 << q
        # Gray: nearest neighbours on the grid differ in exactly one bit
        step = np.min(np.abs(pts[:, None] - pts[None, :]) + 10 * np.eye(1 << q))
        for a in range(1 << q):
            for b in range(1 << q):
                if a != b and abs(abs(pts[a] - pts[b]) - step) < 1e-12:
                    assert np.sum(lab[a] != lab[b]) == 1
        # the transmitter's independent mapping lands on the same labelled points
        np.testing.assert_allclose(synth.qam_map(lab, q), pts, atol=1e-15)


def test_qpsk_and_16qam_closed_form_llrs():
    rng = np.random.default_rng(9)
    x = crandn(rng, (1, 50, 40), 1.5)
    nu = rng.uniform(0.05, 2.0, (1, 40))
    llr = O.demod_stage(x, nu, 2)
    s2 = 2 * math.sqrt(2)
    np.testing.assert_allclose(llr[..., 0], s2 * x.real / nu[:, None, :], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(llr[..., 1], s2 * x.imag / nu[:, None, :], rtol=1e-12, atol=1e-12)
    d = 1 / math.sqrt(10)
    llr = O.demod_stage(x, nu, 4)
    for ax, (bo, bi) in ((x.real, (0, 2)), (x.imag, (1, 3))):
        a = np.abs(ax)
        outer = np.where(a <= 2 * d, 4 * d * ax, 8 * d * (ax - d * np.sign(ax)))
        np.testing.assert_allclose(llr[..., bo], outer / nu[:, None, :], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(llr[..., bi], 4 * d * (2 * d - a) / nu[:, None, :], rtol=1e-12, atol=1e-12)


def test_64qam_points_decode_to_their_labels():
    pts, lab = O.constellation(6)
    llr = O.demod_stage(pts[None, None, :], np.ones((1, 64)), 6)
    assert np.array_equal(O.hard_bits(llr[0, 0]), lab.astype(np.uint8))
    assert np.all(np.abs(llr) > 0)


def test_zf_maxlog_equals_ml_maxlog_for_one_user():
    rng = np.random.default_rng(10)
    for q in (2, 4, 6):
        h = crandn(rng, (4, 1))
        y = crandn(rng, (4,))
        n0 = 0.4
        ml = O.ml_maxlog(h, y, n0, q)
        o = O.detect_stage(h[:, :, None], y[:, None, None], n0, O.ZF)
        zf = O.demod_stage(o["xt"], o["nu"], q)[0, 0, 0]
        np.testing.assert_allclose(zf, ml[0], rtol=1e-10, atol=1e-10)


def test_two_by_two_zf_vs_ml():
    rng = np.random.default_rng(11)
    pts, lab = O.constellation(2)
    n_re, errs_zf, errs_ml = 10000, 0, 0
    for t in range(n_re):
        H = crandn(rng, (2, 2))
        idx = rng.integers(0, 4, 2)
        s = pts[idx]
        y = H @ s
        if t < 50:   # noiseless: both recover the transmitted bits
            o = O.detect_stage(H[:, :, None], y[:, None, None], 1.0, O.ZF)
            zb = O.hard_bits(O.demod_stage(o["xt"], o["nu"], 2))[:, 0, 0]
            mb = O.hard_bits(O.ml_maxlog(H, y, 1.0, 2))
            assert np.array_equal(zb, lab[idx]) and np.array_equal(mb, lab[idx])
        n0 = 10 ** (-20 / 10) * 2      # ~17 dB per receive antenna
        y = y + crandn(rng, (2,), math.sqrt(n0))
        o = O.detect_stage(H[:, :, None], y[:, None, None], n0, O.ZF)
        zb = O.hard_bits(O.demod_stage(o["xt"], o["nu"], 2))[:, 0, 0]
        mb = O.hard_bits(O.ml_maxlog(H, y, n0, 2))
        errs_zf += int(np.sum(zb != lab[idx]))
        errs_ml += int(np.sum(mb != lab[idx]))
    assert errs_ml > 0 and errs_zf >= errs_ml


# ---------------------------------------------------------------------- adjoint
def inner(a, b):
    return np.sum(np.conj(a) * b)


def test_fft_and_csi_adjoint_identities():
    rng = np.random.default_rng(12)
    N, n_sc, cp = 128, 70, 6
    v = crandn(rng, (3, 2, cp + N))
    w = crandn(rng, (3, 2, n_sc))
    lhs = inner(O.fft_stage(v, N, n_sc, cp), w)
    rhs = inner(v, O.fft_adjoint(w, N, n_sc, cp))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) * 10
    M, K, n_sc = 4, 3, 20                       # 20 = 6*3 + 2 trailing
    p = crandn(rng, (n_sc,))
    v = crandn(rng, (M, n_sc))
    w = crandn(rng, (M, K, n_sc))
    lhs = inner(O.csi_stage(v, p, K), w)
    rhs = inner(v, O.csi_adjoint(w, p, n_sc))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) * 10


@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_detect_adjoint_matches_torch_autograd(det):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    M, K, D, n_sc, n0 = 9, 4, 5, 6, 0.6
    H = rand_channel(rng, n_sc, M, K, scale=np.array([1.0, 2.0, 0.7, 1.3]))
    Y = crandn(rng, (M, D, n_sc))
    gx = crandn(rng, (K, D, n_sc))
    gn = rng.standard_normal((K, n_sc))
    gH, gY = O.detect_adjoint(H, Y, n0, det, gx, gn)
    # an independent differentiable forward with library solves, in float64
    Ht = torch.tensor(np.moveaxis(H, -1, 0), requires_grad=True)
    Yt = torch.tensor(np.moveaxis(Y, -1, 0), requires_grad=True)
    A = Ht.conj().transpose(-1, -2) @ Ht
    if det == O.MMSE:
        A = A + n0 * torch.eye(K, dtype=A.dtype)
    xh = torch.linalg.solve(A, Ht.conj().transpose(-1, -2) @ Yt)
    dd = torch.diagonal(torch.linalg.inv(A), dim1=-2, dim2=-1).real
    if det == O.MMSE:
        mu = 1 - n0 * dd
        xt = xh / mu[..., None]
        nu = (1 - mu) / mu
    else:
        xt, nu = xh, n0 * dd
    loss = (torch.real(torch.sum(torch.tensor(np.moveaxis(gx, -1, 0)).conj() * xt))
            + torch.sum(torch.tensor(gn.T) * nu))
    loss.backward()
    np.testing.assert_allclose(gH, np.moveaxis(Ht.grad.numpy(), 0, -1), rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(gY, np.moveaxis(Yt.grad.numpy(), 0, -1), rtol=1e-9, atol=1e-10)


def test_bce_loss_value_and_gradient():
    """The loss of the differentiation workload: mean binary cross-entropy with
    logit(bit = 1) = -LLR.  Pinned by closed forms (LLR 0 gives ln 2 and
    gradient (bit - 1/2)/n; a confident right decision costs about 0 and a
    confident wrong one |LLR|/n) and by torch's own BCE-with-logits and its
    autograd gradient, in float64 on the CPU."""
    torch = pytest.importorskip("torch")
    n = 8
    bits = np.array([0, 1, 0, 1, 1, 0, 0, 1], dtype=np.uint8)
    loss, g = O.bce_loss(np.zeros(n), bits)
    assert loss == pytest.approx(math.log(2), rel=1e-15)
    np.testing.assert_allclose(g, (bits - 0.5) / n, rtol=0, atol=1e-17)
    # LLR = +40 says bit 0: right for bit 0 (cost ~ e^-40), wrong for bit 1 (cost ~ 40)
    l_right, _ = O.bce_loss(np.array([40.0]), np.array([0]))
    l_wrong, g_wrong = O.bce_loss(np.array([40.0]), np.array([1]))
    assert l_right == pytest.approx(math.exp(-40), rel=1e-12)
    assert l_wrong == pytest.approx(40 + math.exp(-40), rel=1e-15)
    assert g_wrong[0] == pytest.approx(1.0 / (1.0 + math.exp(-40)), rel=1e-15)  # d/dLLR of -log(sigmoid(-LLR))
    rng = np.random.default_rng(31)
    llr = rng.standard_normal((3, 5, 7, 4)) * 8.0
    llr[0, 0, 0, 0] = 750.0                      # exp overflow territory for a naive form
    llr[0, 0, 0, 1] = -750.0
    bits = rng.integers(0, 2, llr.shape).astype(np.uint8)
    loss, g = O.bce_loss(llr, bits)
    lt = torch.tensor(llr, requires_grad=True)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(-lt, torch.tensor(bits, dtype=torch.float64))
    ref.backward()
    assert loss == pytest.approx(float(ref), rel=1e-13)
    np.testing.assert_allclose(g, lt.grad.numpy(), rtol=1e-12, atol=1e-18)


def test_torch_gradient_convention():
    torch = pytest.importorskip("torch")
    z = torch.tensor(1 + 1j, dtype=torch.complex128, requires_grad=True)
    (z.abs() ** 2).backward()
    assert complex(z.grad) == pytest.approx(2 + 2j)


def _loss_of_x(x, fr, sh, n0, det):
    o = O.forward(x, fr.pilots, sh, n0, det)
    return O.bce_loss(o["llr"], fr.bits)[0], o


def _argmin_pattern(o, q):
    pts, lab = O.constellation(q)
    dist = np.abs(o["xt"][..., None] - pts) ** 2
    return np.argmin(dist, axis=-1)


@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_full_adjoint_vs_central_differences(det):
    sh = synth.Shape(6, 2, 64, 40, 14, 3, 4)
    fr = synth.make_frame(5, 0, shape=sh, snr=(8.0, 12.0))
    n0 = 1.0
    x = fr.x.astype(np.complex128)
    L0, o0 = _loss_of_x(x, fr, sh, n0, det)
    _, dllr = O.bce_loss(o0["llr"], fr.bits)
    gx, _ = O.backward(x, fr.pilots, sh, n0, det, dllr)
    assert np.all(gx[..., :sh.cp_len] == 0)
    rng = np.random.default_rng(14)
    h = 1e-4
    base = _argmin_pattern(o0, sh.qam_bits)
    checked = 0
    for _ in range(32):
        m, s, n = rng.integers(sh.M), rng.integers(sh.n_sym), rng.integers(sh.cp_len, sh.sym_len)
        for part in (1.0, 1j):
            e = np.zeros_like(x)
            e[m, s, n] = part * h
            Lp, op = _loss_of_x(x + e, fr, sh, n0, det)
            Lm, om = _loss_of_x(x - e, fr, sh, n0, det)
            if not (np.array_equal(_argmin_pattern(op, sh.qam_bits), base)
                    and np.array_equal(_argmin_pattern(om, sh.qam_bits), base)):
                continue
            fd = (Lp - Lm) / (2 * h)
            an = gx[m, s, n].real if part == 1.0 else gx[m, s, n].imag
            assert fd == pytest.approx(an, rel=1e-5, abs=1e-9 * max(1.0, abs(L0)))
            checked += 1
    assert checked >= 48
    # a random direction over every sample
    v = (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    Lp, _ = _loss_of_x(x + h * v, fr, sh, n0, det)
    Lm, _ = _loss_of_x(x - h * v, fr, sh, n0, det)
    fd = (Lp - Lm) / (2 * h)
    assert fd == pytest.approx(np.real(np.sum(np.conj(gx) * v)), rel=1e-5)


def test_cascaded_theta_gradient_vs_central_differences():
    rng = np.random.default_rng(15)
    sh = synth.Shape(8, 2, 64, 40, 14, 0, 4)
    n_el = 16
    Gm, Fm, Hd = crandn(rng, (sh.M, n_el)), crandn(rng, (n_el, sh.K)), crandn(rng, (sh.M, sh.K))
    theta = rng.uniform(0, 2 * np.pi, n_el)
    amp = np.sqrt(10 ** (np.array([12.0, 15.0]) / 10))
    bits = rng.integers(0, 2, (sh.K, sh.n_data, sh.n_sc, 4)).astype(np.uint8)
    sym = synth.qam_map(bits, 4)
    pil = synth.qam_map(rng.integers(0, 2, (sh.n_sc, 2)), 2)
    noise = crandn(rng, (sh.M, sh.n_sym, sh.n_fft), math.sqrt(1.0 / sh.n_fft))

    def xof(th):
        H = synth.frames.cascaded_channel(th, Gm, Fm, Hd)
        he = np.broadcast_to((H * amp[None, :])[:, :, None], (sh.M, sh.K, sh.n_sc))
        return synth.frames.synthesize(sh, he, sym, pil, noise)

    def loss(th):
        o = O.forward(xof(th), pil, sh, 1.0, O.MMSE)
        return O.bce_loss(o["llr"], bits)

    L0, dllr = loss(theta)
    gx, _ = O.backward(xof(theta), pil, sh, 1.0, O.MMSE, dllr)
    gth = O.cascaded_theta_grad(gx, sh, theta, Gm, Fm, amp, sym, pil)
    h = 1e-4
    for k in range(n_el):
        e = np.zeros(n_el)
        e[k] = h
        fd = (loss(theta + e)[0] - loss(theta - e)[0]) / (2 * h)
        assert fd == pytest.approx(gth[k], rel=1e-4, abs=1e-8)
    v = rng.standard_normal(n_el)
    fd = (loss(theta + h * v)[0] - loss(theta - h * v)[0]) / (2 * h)
    assert fd == pytest.approx(gth @ v, rel=1e-4)


# ------------------------------------------------------------ generator sanity
def test_generator_seeded_and_shaped():
    a = synth.make_frame(1, 0)
    b = synth.make_frame(1, 0)
    assert np.array_equal(a.x, b.x) and a.x.dtype == np.complex64
    sh = a.shape
    assert a.x.shape == (sh.M, sh.n_sym, sh.cp_len + sh.n_fft)
    assert a.bits.shape == (sh.K, sh.n_data, sh.n_sc, sh.qam_bits)
    c = synth.make_frame(1, 1)
    assert not np.array_equal(a.x, c.x)
    shapes = synth.draw_batch_shapes(256)
    assert all(s.n_fft >= 1.2 * s.n_sc and s.n_fft < 2.4 * s.n_sc for s in shapes)
    assert all(1 <= s.K <= min(16, s.M) for s in shapes)
    assert {s.M for s in shapes} == {8, 16, 32, 64} and {s.qam_bits for s in shapes} == {2, 4, 6}


def test_snr_definition():
    sh = synth.Shape(32, 2, 256, 200, 14, 0, 2)
    fr = synth.make_frame(9, 0, shape=sh, snr=(20.0, 20.0))
    # received data power per antenna per RE equals sum_u P_u * E|h|^2 (= 2 * 100)
    yf = O.fft_stage(fr.x, sh.n_fft, sh.n_sc)
    p = np.mean(np.abs(yf[:, 1:, :]) ** 2) - fr.n0
    assert p == pytest.approx(200.0, rel=0.2)


def test_torch_cascade_synthesis_matches_frames_and_oracle_theta_grad():
    torch = pytest.importorskip("torch")
    from synth.torch_cascade import cascaded_x
    sh = synth.Shape(8, 2, 128, 60, 14, 0, 4)
    fr = synth.make_frame(5, 0, shape=sh, keep_noise=True)
    th = torch.tensor(fr.extra["theta"], dtype=torch.float64, requires_grad=True)
    x = cascaded_x(th, fr, device="cpu")
    np.testing.assert_allclose(x.detach().numpy()[0], fr.x, atol=1e-6)
    # the generator's own adjoint (autograd) agrees with the oracle's hand-written one
    rng = np.random.default_rng(16)
    gx = (rng.standard_normal(fr.x.shape) + 1j * rng.standard_normal(fr.x.shape))
    L = torch.real(torch.sum(torch.tensor(np.conj(gx)[None], dtype=torch.complex128) * x.to(torch.complex128)))
    L.backward()
    ref = O.cascaded_theta_grad(gx, sh, fr.extra["theta"], fr.extra["G"], fr.extra["F"],
                                fr.extra["amp"], fr.symbols, fr.pilots)
    np.testing.assert_allclose(th.grad.numpy(), ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())


# ---------------------------------------------------------------------- downlink
@pytest.mark.parametrize("q", [2, 4, 6])
def test_modulate_labels_generator_and_noiseless_round_trip(q):
    """modulate_stage puts each label on its constellation point, agrees with
    the generator's independent mapping, and noiseless max-log demapping of
    its output returns the bits."""
    rng = np.random.default_rng([7, q])
    bits = rng.integers(0, 2, (3, 5, 11, q))
    s = O.modulate_stage(bits, q)
    assert np.allclose(s, synth.qam_map(bits, q), atol=1e-15, rtol=0)
    pts, lab = O.constellation(q)
    assert np.array_equal(O.modulate_stage(lab, q), pts)
    llr = O.demod_stage(s.reshape(3, 55), np.ones((3, 55)), q)
    assert np.array_equal(O.hard_bits(llr).reshape(bits.shape), bits)


def _well_conditioned(rng, M, K, n_sc):
    return (rng.standard_normal((M, K, n_sc)) + 1j * rng.standard_normal((M, K, n_sc))) / math.sqrt(2)


@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_precoder_matches_explicit_inverse_and_zf_loopback(det):
    """X = H (H^H H [+ N0 I])^-1 S, checked against numpy's inverse of A
    (a different method); for ZF the downlink channel H^H returns S."""
    rng = np.random.default_rng(11)
    M, K, D, n_sc, n0 = 8, 4, 3, 6, 0.7
    H = _well_conditioned(rng, M, K, n_sc)
    S = rng.standard_normal((K, D, n_sc)) + 1j * rng.standard_normal((K, D, n_sc))
    out = O.precode_stage(H, S, n0, det)
    assert not out["flags"].any()
    for i in range(n_sc):
        A = H[:, :, i].conj().T @ H[:, :, i] + (n0 * np.eye(K) if det == O.MMSE else 0)
        ref = H[:, :, i] @ np.linalg.inv(A) @ S[:, :, i]
        assert np.allclose(out["x"][:, :, i], ref, rtol=1e-12, atol=1e-12)
        if det == O.ZF:
            assert np.allclose(H[:, :, i].conj().T @ out["x"][:, :, i], S[:, :, i], rtol=1e-12, atol=1e-12)


def test_precoder_single_user_closed_form():
    """K = 1: x = h s / |h|^2 (maximum-ratio direction, unit gain back)."""
    rng = np.random.default_rng(12)
    h = rng.standard_normal((5, 1, 4)) + 1j * rng.standard_normal((5, 1, 4))
    s = rng.standard_normal((1, 2, 4)) + 1j * rng.standard_normal((1, 2, 4))
    x = O.precode_stage(h, s)["x"]
    ref = h[:, 0, None, :] * s[0][None] / np.sum(np.abs(h[:, 0, :]) ** 2, axis=0)[None, None, :]
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-14)


def test_precoder_breakdown_and_nonfinite():
    rng = np.random.default_rng(13)
    H = _well_conditioned(rng, 6, 3, 3)
    H[:, 2, 1] = H[:, 0, 1]                         # rank deficient on subcarrier 1
    H[4, 1, 2] = np.nan                             # non-finite on subcarrier 2
    out = O.precode_stage(H, np.ones((3, 2, 3), dtype=np.complex128))
    assert out["flags"][0] == 0
    assert out["flags"][1] == O.FLAG_BREAKDOWN and out["flags"][2] == O.FLAG_NONFINITE
    assert not out["x"][:, :, 1:].any()


@pytest.mark.parametrize("N,n_sc,cp", [(8, 5, 2), (16, 16, 0), (64, 37, 9)])
def test_ifft_stage_definition_cp_and_inverse(N, n_sc, cp):
    """Term by term e^{+j 2 pi bin(i) n / N}; the prefix is the tail; and the
    forward stage undoes it up to the factor N."""
    rng = np.random.default_rng([14, N])
    X = rng.standard_normal((2, n_sc)) + 1j * rng.standard_normal((2, n_sc))
    x = O.ifft_stage(X, N, n_sc, cp)
    bins = O.used_bins(N, n_sc)
    for n in range(N):
        ref = sum(X[:, i] * np.exp(2j * math.pi * bins[i] * n / N) for i in range(n_sc))
        assert np.allclose(x[:, cp + n], ref, rtol=1e-12, atol=1e-12)
    assert np.array_equal(x[:, :cp], x[:, N:N + cp])
    assert np.allclose(O.fft_stage(x, N, n_sc, cp), N * X, rtol=1e-12, atol=1e-11)
