"""Mixed-precision detector (BF16 / FP16 products on MFMA, FP32 Cholesky, FP64
refinement of subcarriers whose condition estimate exceeds the threshold)
against the FP64 oracle on the same FP32 inputs.  Apart from the bounds below,
the errors of the unrefined low-precision solution are reported, not asserted
(there is no exact reference for a rounded product)."""
import numpy as np
import pytest

import oracle as O
import synth
from parity_util import evm_rel, hard_bits_outside_guard, llr_rel, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-mixed]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _inputs(rx, sh, cfg, nfr, channel=None, snr=None, det=O.ZF):
    frs = [synth.make_frame(cfg, f, shape=sh, channel=channel, snr=snr) for f in range(nfr)]
    fr = rx.Frame.of(sh, det, 1.0)
    x = dev(np.stack([f.x for f in frs]))
    p = dev(np.stack([f.pilots for f in frs]))
    yf = rx.fft(fr, x)
    h = rx.csi(fr, yf, p)
    return fr, frs, yf, h


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("det", [O.ZF, O.MMSE])
@pytest.mark.parametrize("K", [12, 16])        # 16: tiles share one channel matrix
def test_refine_everything_equals_fp64_solution(rx, prec, det, K):
    sh = synth.Shape(32, K, 1024, 601, 14, 0, 4)
    fr, frs, yf, h = _inputs(rx, sh, 31, 2, snr=(5, 25), det=det)
    xt, nu, fl = (host(t) for t in rx.detect(fr, h, yf, prec, 0.0))
    yfh, hh = host(yf), host(h)
    for f in range(2):
        ref = O.detect_stage(hh[f], yfh[f, :, 1:, :], 1.0, det, want_kappa=True)
        assert np.all(fl[f] == O.FLAG_REFINED)
        e = evm_rel(xt[f], ref["xt"], np.ones(sh.n_sc, bool))
        en = rel_rms(nu[f], ref["nu"])
        say(prec, det, "refined-all evm_rel", e, "nu_rel", en)
        assert e < 1e-6 and en < 1e-6


@pytest.mark.parametrize("prec,bound", [("bf16", 0.1), ("fp16", 0.02)])
def test_unrefined_error_scales_with_precision(rx, prec, bound):
    sh = synth.Shape(64, 16, 2048, 1200, 14, 0, 4)
    fr, frs, yf, h = _inputs(rx, sh, 2, 1)
    xt, nu, fl = (host(t) for t in rx.detect(fr, h, yf, prec, float("inf")))
    x32, nu32, _ = (host(t) for t in rx.detect(fr, h, yf, "fp32"))
    ref = O.detect_stage(host(h)[0], host(yf)[0, :, 1:, :], 1.0, O.ZF, want_kappa=True)
    good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
    e = evm_rel(xt[0], ref["xt"], good)
    e32 = evm_rel(x32[0], ref["xt"], good)
    say(prec, "no refinement: evm_rel", e, "(fp32:", e32, ") kappa max", float(ref["kappa"].max()))
    assert np.all(fl == 0)
    assert e32 < e < bound


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_ill_conditioned_subcarriers_are_refined(rx, prec):
    # users 0 and 1 nearly collinear on every odd subcarrier (kappa ~ 1e5),
    # independent Rayleigh columns on the even ones (kappa ~ 10)
    rng = np.random.default_rng(33)
    M, K, n_sc, S = 16, 4, 96, 6
    base = (rng.standard_normal((1, M, K, n_sc)) + 1j * rng.standard_normal((1, M, K, n_sc))) / np.sqrt(2)
    base[:, :, 1, :] = base[:, :, 0, :] + 3e-3 * (rng.standard_normal((1, M, n_sc)) + 1j * rng.standard_normal((1, M, n_sc)))
    base[:, :, :, ::2] = (rng.standard_normal((1, M, K, n_sc // 2)) + 1j * rng.standard_normal((1, M, K, n_sc // 2))) / np.sqrt(2)
    h = (base * 10).astype(np.complex64)
    yf = ((rng.standard_normal((1, M, S, n_sc)) + 1j * rng.standard_normal((1, M, S, n_sc))) * 10).astype(np.complex64)
    fr = rx.Frame(M, K, 512, n_sc, S, 0, 4, O.ZF, 1.0)
    xt, nu, fl = (host(t) for t in rx.detect(fr, dev(h), dev(yf), prec, 1e3))
    ref = O.detect_stage(h[0], yf[0, :, 1:, :], 1.0, O.ZF, want_kappa=True)
    refined = fl[0] == O.FLAG_REFINED
    say(prec, "refined", int(refined.sum()), "of", n_sc, "kappa range", float(ref["kappa"].min()), float(ref["kappa"].max()))
    assert np.all(refined[1::2])                      # the collinear subcarriers
    # the estimate ||A||_F tr(A^-1) never falls below kappa_2 and exceeds it by
    # at most K^1.5: no subcarrier above the threshold escapes, and none below
    # threshold / K^1.5 is refined
    assert np.all(refined[ref["kappa"] > 1e3])
    assert np.all(ref["kappa"][refined] > 1e3 / K ** 1.5)
    e = evm_rel(xt[0], ref["xt"], refined)
    say("  refined evm_rel", e)
    assert e < 1e-5
    assert rel_rms(nu[0][:, refined], ref["nu"][:, refined]) < 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_low_precision_breakdown_is_solved_in_fp64(rx, prec):
    """Users 0 and 1 get channel columns that differ only below the operand
    precision: column 0 holds values exact in BF16 (so in FP16 too) and
    column 1 = column 0 (1 + 2e-4 r), |r| <= 1, which rounds back to column 0.  The
    low-precision Gram matrix is then exactly rank deficient and its FP32
    Cholesky factor breaks down or nearly does, while the FP64 factor of the
    FP32 inputs exists (kappa ~ 1e8-1e9).  Every such subcarrier must come
    back REFINED with finite outputs equal to the FP64 solution."""
    rng = np.random.default_rng(35)
    M, K, n_sc, S = 16, 4, 64, 6
    h = (rng.standard_normal((1, M, K, n_sc)) + 1j * rng.standard_normal((1, M, K, n_sc))) * 4
    c0 = np.ascontiguousarray(h[:, :, 0, :]).astype(np.complex64)
    t = torch.from_numpy(c0.view(np.float32).copy())
    c0 = t.to(torch.bfloat16).to(torch.float32).numpy().view(np.complex64).astype(np.complex128)
    h[:, :, 0, :] = c0
    h[:, :, 1, :] = c0 * (1 + 2e-4 * rng.uniform(-1, 1, c0.shape))
    h = h.astype(np.complex64)
    yf = ((rng.standard_normal((1, M, S, n_sc)) + 1j * rng.standard_normal((1, M, S, n_sc))) * 10).astype(np.complex64)
    fr = rx.Frame(M, K, 512, n_sc, S, 0, 4, O.ZF, 1.0)
    xt, nu, fl = (host(t) for t in rx.detect(fr, dev(h), dev(yf), prec, 1e3))
    ref = O.detect_stage(h[0], yf[0, :, 1:, :], 1.0, O.ZF, want_kappa=True)
    say(prec, "kappa range", float(ref["kappa"].min()), float(ref["kappa"].max()), "oracle flags",
        int(np.sum(ref["flags"] != 0)))
    assert np.all(ref["flags"] == 0)                  # FP64 factors every subcarrier
    assert np.all(fl[0] == O.FLAG_REFINED)
    assert np.all(np.isfinite(xt)) and np.all(np.isfinite(nu))
    e = evm_rel(xt[0], ref["xt"], np.ones(n_sc, bool))
    en = rel_rms(nu[0], ref["nu"])
    say("  evm_rel", e, "nu_rel", en)
    assert e < 1e-5 and en < 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_kronecker_64qam_workload_report(rx, prec):
    """64x16, N 4096, 3276 subcarriers, 64-QAM, Kronecker (0.7, 0.3), 25 dB."""
    sh = synth.config_shape(3)
    fr, frs, yf, h = _inputs(rx, sh, 3, 1)
    xt, nu, fl = rx.detect(fr, h, yf, prec, 1e3)
    llr = host(rx.demod(fr, xt, nu))[0]
    xt, nu, fl = host(xt)[0], host(nu)[0], host(fl)[0]
    ref = O.forward(frs[0].x, frs[0].pilots, sh, 1.0, O.ZF, want_kappa=True)
    good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
    e = evm_rel(xt, ref["xt"], good)
    lrel = llr_rel(llr, ref["llr"])
    tau = float(np.max(np.abs(llr - ref["llr"])))
    mism, band = hard_bits_outside_guard(llr, ref["llr"])
    # first-order perturbation: relative LLR error <~ kappa * unit roundoff of
    # the product precision, so hard bits must agree outside that band
    u = 2.0 ** -8 if prec == "bf16" else 2.0 ** -11
    kap = float(ref["kappa"][good].max())
    mism_p, band_p = hard_bits_outside_guard(llr, ref["llr"], rel_tau=u * kap)
    ber_gpu = float(np.mean(O.hard_bits(llr) != frs[0].bits))
    ber_ref = float(np.mean(O.hard_bits(ref["llr"]) != frs[0].bits))
    say(prec, "evm_rel", e, "llr_rel", lrel, "max |dLLR|", tau, "refined", int(np.sum(fl == O.FLAG_REFINED)),
        "hard-bit mismatches outside the 1e-5 band", mism, "outside the kappa*u band", mism_p,
        "(", band_p, "bits inside ) BER", ber_gpu, "vs FP64", ber_ref)
    assert mism_p == 0
    assert np.all(fl[ref["kappa"] > 1e3] == O.FLAG_REFINED)
    assert np.all(ref["kappa"][fl == O.FLAG_REFINED] > 1e3 / 16 ** 1.5)
    assert abs(ber_gpu - ber_ref) < 0.1 * ber_ref + 1e-4
