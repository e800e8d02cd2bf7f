"""GPU adjoint (rxphy_backward) against the FP64 oracle's hand-written adjoint
and against central finite differences of the FP64 oracle forward."""
import math

import numpy as np
import pytest

import oracle as O
import synth
from parity_util import elem_rel, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-backward]", *a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


BWD_CASES = [
    # M, K, N, n_sc, cp, Q, detector, snr
    (8, 2, 512, 300, 0, 2, O.ZF, (20, 20)),
    (8, 2, 512, 300, 36, 4, O.MMSE, (10, 15)),
    (12, 5, 512, 77, 7, 6, O.MMSE, (15, 25)),
    (16, 16, 512, 64, 0, 4, O.ZF, (25, 25)),
    (64, 16, 2048, 1200, 0, 4, O.MMSE, (10, 30)),
    (64, 8, 1024, 601, 0, 2, O.ZF, (10, 20)),
    # the CSI adjoint's butterfly forms: one user, and pilot groups that leave
    # a tail past G K (K = 4: 203 = 50 x 4 + 3; K = 16: 70 = 4 x 16 + 6)
    (8, 1, 512, 131, 0, 2, O.ZF, (20, 20)),
    (16, 4, 512, 203, 0, 4, O.MMSE, (15, 20)),
    (32, 16, 512, 70, 0, 2, O.ZF, (25, 25)),
]


# slots of other lengths than 14 symbols (the apply kernel's generic symbol
# bound, with 4, 8 and 16 padded users): 5, 8, 11 and the longest, 17 symbols
BWD_SLOT_CASES = [
    # M, K, N, n_sc, n_sym, cp, Q, detector, snr
    (16, 4, 512, 150, 8, 0, 4, O.MMSE, (15, 20)),
    (32, 16, 512, 96, 17, 0, 2, O.ZF, (25, 25)),
    (8, 3, 512, 100, 5, 4, 2, O.ZF, (20, 20)),
    (12, 6, 512, 90, 11, 0, 4, O.MMSE, (15, 25)),
]


@pytest.mark.parametrize("M,K,N,n_sc,n_sym,cp,Q,det,snr", BWD_SLOT_CASES)
def test_backward_other_slot_lengths(rx, M, K, N, n_sc, n_sym, cp, Q, det, snr):
    test_backward_matches_oracle_adjoint(rx, M, K, N, n_sc, cp, Q, det, snr, n_sym=n_sym)


@pytest.mark.parametrize("M,K,N,n_sc,cp,Q,det,snr", BWD_CASES)
def test_backward_matches_oracle_adjoint(rx, M, K, N, n_sc, cp, Q, det, snr, n_sym=14):
    say("backward", M, K, N, n_sc, n_sym, cp, Q, det)
    sh = synth.Shape(M, K, N, n_sc, n_sym, cp, Q)
    fo = synth.make_frame(21, 0, shape=sh, snr=snr)
    rng = np.random.default_rng(M * 1000 + n_sc)
    dllr = rng.standard_normal((1, K, sh.n_data, n_sc, Q)).astype(np.float32)
    fr = rx.Frame.of(sh, det, 1.0)
    x, p = dev(fo.x[None]), dev(fo.pilots[None])
    dx, dh = rx.backward(fr, x, p, dev(dllr), want_dh=True)
    dx, dh = host(dx)[0], host(dh)[0]
    gx, gH = O.backward(fo.x, fo.pilots, sh, 1.0, det, dllr[0].astype(np.float64))
    ex, eh = rel_rms(dx, gx), rel_rms(dh, gH)
    say("  dx rel rms", ex, "dh rel rms", eh)
    assert np.all(dx[..., :cp] == 0)
    assert ex < 1e-3 and eh < 1e-3
    # element-wise, |d - ref| / max(|ref|, 0.01 RMS(ref)) <= 1e-3 on every
    # sample and channel gradient, with the gradient restricted to the
    # subcarriers whose exact kappa_2(A) <= 1e3 (the gate of the EVM bound:
    # the adjoint applies A^{-1} twice, so FP32 errors there grow like
    # kappa^2 u).  Zeroing dL/dLLR on the others removes their contribution
    # exactly (their channel and data gradients are then 0 in both).
    kap = O.forward(fo.x, fo.pilots, sh, 1.0, det, want_kappa=True)["kappa"]
    good = kap <= 1e3
    wx_all, wh_all = elem_rel(dx, gx), elem_rel(dh, gH)
    if not np.all(good):
        dllr = dllr * good[None, None, None, :, None]
        dx, dh = rx.backward(fr, x, p, dev(dllr), want_dh=True)
        dx, dh = host(dx)[0], host(dh)[0]
        gx, gH = O.backward(fo.x, fo.pilots, sh, 1.0, det, dllr[0].astype(np.float64))
        assert np.all(dh[..., ~good] == 0)
    wx, wh = elem_rel(dx, gx), elem_rel(dh, gH)
    say("  %d of %d subcarriers with kappa > 1e3 (max %.3g); element-wise: all subcarriers dx %.3g dh %.3g, "
        "kappa <= 1e3 dx %.3g dh %.3g" % (int(np.sum(~good)), n_sc, float(kap.max()), wx_all, wh_all, wx, wh))
    assert wx < 1e-3 and wh < 1e-3


def test_backward_saved_equals_recomputed(rx):
    sh = synth.Shape(16, 4, 512, 200, 14, 0, 4)
    fo = synth.make_frame(22, 0, shape=sh)
    fr = rx.Frame.of(sh, O.MMSE, 1.0)
    x, p = dev(fo.x[None]), dev(fo.pilots[None])
    out = rx.forward(fr, x, p)
    dllr = torch.randn_like(out["llr"])
    a = rx.backward(fr, x, p, dllr)
    b = rx.backward(fr, x, p, dllr, saved=dict(yf=out["yf"], h=out["h"]))
    c = rx.backward(fr, x, p, dllr, saved=dict(yf=out["yf"], h=out["h"], xt=out["xt"], nu=out["nu"]))
    d = rx.backward(fr, x, p, dllr, saved=dict(xt=out["xt"]))        # xt without nu: recomputed
    assert torch.equal(a, b) and torch.equal(a, c) and torch.equal(a, d)


def _bce(llr, bits):
    return torch.nn.functional.binary_cross_entropy_with_logits(-llr, bits.to(llr.dtype))


def _oracle_loss(x64, fo, det):
    o = O.forward(x64, fo.pilots, fo.shape, 1.0, det)
    return O.bce_loss(o["llr"], fo.bits)[0], o


def _pattern(o, q):
    pts, _ = O.constellation(q)
    return np.argmin(np.abs(o["xt"][..., None] - pts) ** 2, axis=-1)


def test_cascaded_gradients_vs_finite_differences(rx):
    """64x8, N 2048, 1200 subcarriers, 16-QAM, cascaded channel with 256 phases,
    5 dB, MMSE, mean BCE of the max-log LLRs: dL/dx and dL/dtheta from the GPU
    adjoint against central differences (h = 1e-4) of the FP64 oracle."""
    from synth.torch_cascade import cascaded_x
    fo = synth.make_frame(5, 0, keep_noise=True)
    sh = fo.shape
    det = O.MMSE
    fr = rx.Frame.of(sh, det, 1.0)
    bits = dev(fo.bits[None])
    p = dev(fo.pilots[None])
    theta = torch.tensor(fo.extra["theta"], dtype=torch.float64, device="cuda", requires_grad=True)
    x = cascaded_x(theta, fo)
    x.retain_grad()
    llr = rx.RxphyFunction.apply(x, p, fr)
    loss = _bce(llr, bits)
    loss.backward()
    gx = host(x.grad)[0]
    gth = host(theta.grad)
    say("loss", float(loss))

    # dL/dx: FD of the FP64 oracle at the same complex64 samples
    x64 = fo.x.astype(np.complex128)
    L0, o0 = _oracle_loss(x64, fo, det)
    assert abs(L0 - float(loss)) < 1e-4 * abs(L0)
    base = _pattern(o0, sh.qam_bits)
    rng = np.random.default_rng(23)
    h = 1e-4
    fds, ans = [], []
    for _ in range(16):
        m, s, n = rng.integers(sh.M), rng.integers(sh.n_sym), rng.integers(sh.sym_len)
        for part in (1.0, 1j):
            e = np.zeros_like(x64)
            e[m, s, n] = part * h
            Lp, op = _oracle_loss(x64 + e, fo, det)
            Lm, om = _oracle_loss(x64 - e, fo, det)
            if not (np.array_equal(_pattern(op, sh.qam_bits), base) and
                    np.array_equal(_pattern(om, sh.qam_bits), base)):
                continue
            fds.append((Lp - Lm) / (2 * h))
            ans.append(gx[m, s, n].real if part == 1.0 else gx[m, s, n].imag)
    fds, ans = np.array(fds), np.array(ans)
    scale = np.sqrt(np.mean(fds ** 2))
    err = np.max(np.abs(ans - fds) / np.maximum(np.abs(fds), scale))
    say("dL/dx coordinates checked", len(fds), "max rel err", err)
    assert len(fds) >= 24 and err < 1e-3
    v = rng.standard_normal(x64.shape) + 1j * rng.standard_normal(x64.shape)
    fd = (_oracle_loss(x64 + h * v, fo, det)[0] - _oracle_loss(x64 - h * v, fo, det)[0]) / (2 * h)
    dd = float(np.real(np.sum(np.conj(gx) * v)))
    say("dL/dx directional", fd, dd)
    assert abs(dd - fd) < 1e-3 * abs(fd)

    # dL/dtheta: FD through the FP64 synthesis and the FP64 oracle
    def loss_theta(th):
        H = synth.frames.cascaded_channel(th, fo.extra["G"], fo.extra["F"], fo.extra["Hd"])
        he = np.broadcast_to((H * fo.extra["amp"][None, :])[:, :, None], (sh.M, sh.K, sh.n_sc))
        xx = synth.frames.synthesize(sh, he, fo.symbols, fo.pilots.astype(np.complex128), fo.extra["noise_t"])
        return _oracle_loss(xx, fo, det)[0]

    th0 = fo.extra["theta"]
    idx = rng.choice(len(th0), 8, replace=False)
    fdt, ant = [], []
    for k in idx:
        e = np.zeros_like(th0)
        e[k] = h
        fdt.append((loss_theta(th0 + e) - loss_theta(th0 - e)) / (2 * h))
        ant.append(gth[k])
    fdt, ant = np.array(fdt), np.array(ant)
    errt = np.max(np.abs(ant - fdt) / np.maximum(np.abs(fdt), np.sqrt(np.mean(fdt ** 2))))
    say("dL/dtheta FD", fdt[:4], "adjoint", ant[:4], "max rel err", errt)
    assert errt < 1e-3
    vt = rng.standard_normal(len(th0))
    fd = (loss_theta(th0 + h * vt) - loss_theta(th0 - h * vt)) / (2 * h)
    assert abs(float(gth @ vt) - fd) < 1e-3 * abs(fd)
    # and against the oracle's own analytic phase gradient
    _, dllr = O.bce_loss(o0["llr"], fo.bits)
    gx_ref, _ = O.backward(x64, fo.pilots, sh, 1.0, det, dllr)
    gth_ref = O.cascaded_theta_grad(gx_ref, sh, th0, fo.extra["G"], fo.extra["F"], fo.extra["amp"],
                                    fo.symbols, fo.pilots)
    assert rel_rms(gth, gth_ref) < 1e-3
    assert rel_rms(gx, gx_ref) < 1e-3
    eg, et = elem_rel(gx, gx_ref), elem_rel(gth, gth_ref)
    say("dL/dx elem rel", eg, "dL/dtheta elem rel", et)
    assert eg < 1e-3 and et < 1e-3
