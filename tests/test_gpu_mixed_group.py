"""The 16-user fused path (csi + detect, optionally + demod) with BF16 / FP16
operands: the Gram matrix and the matched filter on gfx950's 16x16x32
products, the Cholesky factor and A^-1 Z in FP32, and every pilot group whose
condition estimate ||A||_F tr(A^-1) exceeds the threshold (or whose
low-precision factorisation breaks down) re-solved in FP64 from the FP32
inputs, against the FP64 oracle on the same inputs.  As for the per-subcarrier
mixed detector, the unrefined low-precision errors are bounded, not pinned."""
import numpy as np
import pytest

import oracle as O
import synth
from parity_util import evm_rel, hard_bits_outside_guard, llr_rel, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-mixed-group]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def crandn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def designed_frame(rng, M, n_sc, S, groups_h, data_scale=10.0):
    """yf [1][M][S][n_sc] whose pilot symbol carries the channel of pilot group
    g on subcarrier 16 g + u with unit pilots, so that the LS estimate (FP32 on
    the GPU, FP64 in the oracle) is that channel exactly; the data symbols are
    Gaussian."""
    K = 16
    yf = crandn(rng, (1, M, S, n_sc)) * data_scale
    G = n_sc // K
    for g in range(G):
        yf[0, :, 0, g * K:(g + 1) * K] = groups_h[g]
    p = np.ones((1, n_sc), np.complex64)
    return yf.astype(np.complex64), p


def oracle_detect(yf, p, det):
    H = O.csi_stage(yf[0, :, 0, :], p[0], 16)
    return O.detect_stage(H, yf[0, :, 1:, :].astype(np.complex128), 1.0, det, want_kappa=True)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_group_refine_everything_equals_fp64_solution(rx, prec, det):
    """Threshold 0 refines every pilot group: x_tilde and nu equal the FP64
    solution of the FP32 inputs to FP32 rounding (32 x 16, 601 subcarriers:
    the last tile is ragged and belongs to the last full group)."""
    sh = synth.Shape(32, 16, 1024, 601, 14, 0, 4)
    frs = [synth.make_frame(31, f, shape=sh, snr=(5, 25)) for f in range(2)]
    fr = rx.Frame.of(sh, det, 1.0)
    yf = rx.fft(fr, dev(np.stack([f.x for f in frs])))
    p = dev(np.stack([f.pilots for f in frs]))
    xt, nu, fl = (host(t) for t in rx.csi_detect(fr, yf, p, prec, 0.0))
    llr, nu2, fl2, _ = rx.csi_detect_demod(fr, yf, p, prec, 0.0)
    llr, nu2, fl2 = host(llr), host(nu2), host(fl2)
    yfh, ph = host(yf), host(p)
    for f in range(2):
        ref = oracle_detect(yfh[f:f + 1], ph[f:f + 1], det)
        assert np.all(fl[f] == O.FLAG_REFINED) and np.all(fl2[f] == O.FLAG_REFINED)
        e = evm_rel(xt[f], ref["xt"], np.ones(sh.n_sc, bool))
        en = rel_rms(nu[f], ref["nu"])
        lref = O.demod_stage(ref["xt"], ref["nu"], sh.qam_bits)
        el = llr_rel(llr[f], lref)
        mism, band = hard_bits_outside_guard(llr[f], lref)
        say(prec, det, "refined-all evm_rel", e, "nu_rel", en, "llr_rel", el, "mismatches", mism)
        assert e < 1e-6 and en < 1e-6 and el < 1e-3 and mism == 0
        assert np.array_equal(nu[f], nu2[f])


@pytest.mark.parametrize("prec,bound", [("bf16", 0.1), ("fp16", 0.02)])
def test_group_unrefined_error_scales_with_precision(rx, prec, bound):
    """Threshold infinity on the 64 x 16 workload: no group is refined; the
    error sits between the FP32 path's and the precision's bound."""
    sh = synth.config_shape(2)
    fo = synth.make_frame(2, 0)
    fr = rx.Frame.of(sh, O.ZF, 1.0)
    yf = rx.fft(fr, dev(fo.x[None]))
    p = dev(fo.pilots[None])
    xt, nu, fl = (host(t) for t in rx.csi_detect(fr, yf, p, prec, float("inf")))
    x32, _, _ = (host(t) for t in rx.csi_detect(fr, yf, p, "fp32"))
    ref = oracle_detect(host(yf), host(p), O.ZF)
    good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
    e, e32 = evm_rel(xt[0], ref["xt"], good), evm_rel(x32[0], ref["xt"], good)
    say(prec, "group path, no refinement: evm_rel", e, "(fp32:", e32, ")")
    assert np.all(fl == 0)
    assert e32 < e < bound


def _mixed_groups(rng, M, G, bad_every=2, eps=3e-3):
    hs = []
    for g in range(G):
        h = crandn(rng, (M, 16)) * 3
        if g % bad_every == 1:                            # users 0 and 1 nearly collinear
            h[:, 1] = h[:, 0] + eps * crandn(rng, (M,))
        hs.append(h)
    return hs


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
def test_group_ill_conditioned_groups_are_refined(rx, prec, det):
    """Every other pilot group has two nearly collinear users (kappa ~ 1e5 -
    1e6): those groups, and any other group above the threshold, are refined
    and equal the FP64 solution; groups refined have kappa above
    threshold / 16^1.5 (the estimate's bounds); csi_detect_demod's LLRs are
    the demod stage's LLRs of csi_detect's outputs, bit for bit."""
    rng = np.random.default_rng(41)
    M, S, G = 32, 6, 12
    n_sc = 16 * G + 7                                     # ragged last tile
    yf, p = designed_frame(rng, M, n_sc, S, _mixed_groups(rng, M, G))
    fr = rx.Frame(M, 16, 512, n_sc, S, 0, 4, det, 1.0)
    yfd, pd = dev(yf), dev(p)
    xt, nu, fl = rx.csi_detect(fr, yfd, pd, prec, 1e3)
    llr = rx.demod(fr, xt, nu)
    llr2, nu2, fl2, xt2 = rx.csi_detect_demod(fr, yfd, pd, prec, 1e3, want_xt=True)
    assert torch.equal(llr, llr2) and torch.equal(nu, nu2) and torch.equal(fl, fl2) and torch.equal(xt, xt2)
    xt, nu, fl = host(xt)[0], host(nu)[0], host(fl)[0]
    ref = oracle_detect(yf, p, det)
    refined = fl == O.FLAG_REFINED
    say(prec, det, "refined", int(refined.sum()), "of", n_sc, "kappa range", float(ref["kappa"].min()),
        float(ref["kappa"].max()))
    assert np.all(refined[ref["kappa"] > 1e3])
    assert np.all(ref["kappa"][refined] > 1e3 / 16 ** 1.5)
    assert np.all(fl[~refined] == 0)
    e = evm_rel(xt, ref["xt"], refined)
    en = rel_rms(nu[:, refined], ref["nu"][:, refined])
    say("  refined evm_rel", e, "nu_rel", en)
    assert e < 1e-5 and en < 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_group_low_precision_breakdown_is_solved_in_fp64(rx, prec):
    """Users 0 and 1 of every group have channel columns that coincide after
    BF16 / FP16 rounding (column 0 exact in BF16, column 1 within 2e-4 of it),
    so the low-precision Gram matrix is singular while the FP64 factor of the
    FP32 inputs exists: every group comes back REFINED, finite and equal to
    the FP64 solution."""
    rng = np.random.default_rng(43)
    M, S, G = 32, 6, 6
    n_sc = 16 * G
    hs = []
    for g in range(G):
        h = crandn(rng, (M, 16)) * 3
        c0 = h[:, 0].astype(np.complex64)
        c0 = torch.from_numpy(c0.view(np.float32).copy()).to(torch.bfloat16).to(torch.float32).numpy()
        c0 = c0.view(np.complex64).astype(np.complex128)
        h[:, 0] = c0
        h[:, 1] = c0 * (1 + 2e-4 * rng.uniform(-1, 1, M))
        hs.append(h)
    yf, p = designed_frame(rng, M, n_sc, S, hs)
    fr = rx.Frame(M, 16, 512, n_sc, S, 0, 4, O.ZF, 1.0)
    xt, nu, fl = (host(t)[0] for t in rx.csi_detect(fr, dev(yf), dev(p), prec, 1e3))
    ref = oracle_detect(yf, p, O.ZF)
    say(prec, "kappa range", float(ref["kappa"].min()), float(ref["kappa"].max()))
    assert np.all(ref["flags"] == 0)
    assert np.all(fl == O.FLAG_REFINED)
    assert np.all(np.isfinite(xt)) and np.all(np.isfinite(nu))
    e = evm_rel(xt, ref["xt"], np.ones(n_sc, bool))
    en = rel_rms(nu, ref["nu"])
    say("  evm_rel", e, "nu_rel", en)
    assert e < 1e-5 and en < 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_group_kronecker_64qam_workload_report(rx, prec):
    """64x16, N 4096, 3276 subcarriers, 64-QAM, Kronecker (0.7, 0.3), 25 dB,
    through the fused call with the demapping: hard bits agree with the FP64
    oracle outside the band kappa * u * RMS(LLR) (first-order perturbation of
    the products' rounding), the BER matches, and no group above the threshold
    escapes refinement."""
    sh = synth.config_shape(3)
    fo = synth.make_frame(3, 0)
    fr = rx.Frame.of(sh, O.ZF, 1.0)
    yf = rx.fft(fr, dev(fo.x[None]))
    p = dev(fo.pilots[None])
    llr, nu, fl, xt = rx.csi_detect_demod(fr, yf, p, prec, 1e3, want_xt=True)
    llr, fl, xt = host(llr)[0], host(fl)[0], host(xt)[0]
    ref = O.forward(fo.x, fo.pilots, sh, 1.0, O.ZF, want_kappa=True)
    good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
    e = evm_rel(xt, ref["xt"], good)
    u = 2.0 ** -8 if prec == "bf16" else 2.0 ** -11
    kap = float(ref["kappa"][good].max())
    mism, band = hard_bits_outside_guard(llr, ref["llr"])
    mism_p, band_p = hard_bits_outside_guard(llr, ref["llr"], rel_tau=u * kap)
    ber_gpu = float(np.mean(O.hard_bits(llr) != fo.bits))
    ber_ref = float(np.mean(O.hard_bits(ref["llr"]) != fo.bits))
    say(prec, "evm_rel", e, "llr_rel", llr_rel(llr, ref["llr"]), "refined", int(np.sum(fl == O.FLAG_REFINED)),
        "mismatches outside the 1e-5 band", mism, "outside the kappa*u band", mism_p, "(", band_p,
        "bits inside ) BER", ber_gpu, "vs FP64", ber_ref)
    assert mism_p == 0
    assert np.all(fl[ref["kappa"] > 1e3] == O.FLAG_REFINED)
    assert abs(ber_gpu - ber_ref) < 0.1 * ber_ref + 1e-4
