"""Plain FP64 oracle of the OFDM massive-MIMO uplink receiver.

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Slow on purpose and
written so that each step can be checked against its definition by eye.

Stages (their names are the DSP-stage macros fft, csi, equal, demod that open
the paper's preamble; the paper gives them no further definition):

  fft    Section III-A1 (detection/localisation formulation): a non-overlapping
         N_FFT-point FFT over consecutive I/Q segments; here one segment per
         (antenna, OFDM symbol) after the cyclic prefix, keeping the used bins.
         Section IV-D: samples are 32-bit floating-point I/Q; the oracle
         upcasts them to complex128.
  csi    least-squares channel estimate from comb pilots, held over each pilot
         group (textbook; reading of the stage name).
  equal  zero-forcing / MMSE linear detection via the Gram matrix, a Cholesky
         factorisation and two triangular solves (textbook).
  demod  max-log LLRs over the Gray square-QAM set, by brute force over every
         constellation point (definition of the max-log LLR).

Downlink (the transmit-side macros modul, precode, ifft of the same preamble):
  modulate_stage  bits -> Gray QAM points; precode_stage  zero-forcing
  precoder from the uplink channel estimate; ifft_stage  inverse transform of
  the used bins with a cyclic prefix.

Every floating-point value is complex128 / float64.  Library primitives used
as steps: numpy's FFT and matrix products.  The Cholesky factorisation and
the triangular solves are written out.
"""
from __future__ import annotations

import math

import numpy as np

ZF, MMSE = 0, 1
FLAG_REFINED, FLAG_BREAKDOWN, FLAG_NONFINITE = 1, 2, 4


# --------------------------------------------------------------------------- fft
def used_bins(n_fft: int, n_sc: int) -> np.ndarray:
    """FFT bin of used subcarrier i: (i - floor(n_sc/2)) mod n_fft (centred, DC kept)."""
    return (np.arange(n_sc) - n_sc // 2) % n_fft


def fft_stage(x, n_fft: int, n_sc: int, cp_len: int = 0) -> np.ndarray:
    """Yf[..., s, i] = sum_n x[..., s, cp+n] exp(-j 2 pi bin(i) n / N), unscaled.

    x: [..., n_sym, cp_len + n_fft] complex; returns [..., n_sym, n_sc] complex128.
    """
    seg = np.asarray(x).astype(np.complex128)[..., cp_len:cp_len + n_fft]
    if seg.shape[-1] != n_fft:
        raise ValueError("time axis shorter than cp_len + n_fft")
    spec = np.fft.fft(seg, axis=-1)
    return spec[..., used_bins(n_fft, n_sc)]


# --------------------------------------------------------------------------- csi
def pilot_groups(n_sc: int, K: int) -> np.ndarray:
    """Pilot group of each subcarrier: min(floor(i/K), G-1), G = floor(n_sc/K)."""
    G = n_sc // K
    if G < 1:
        raise ValueError("need n_sc >= K")
    return np.minimum(np.arange(n_sc) // K, G - 1)


def csi_stage(yf0, pilots, K: int) -> np.ndarray:
    """LS estimate from symbol 0, held over the pilot group.

    H[m][u][i] = Yf0[m][q] * conj(p[q]) / |p[q]|^2 with q = g(i)*K + u, the
    subcarrier of group g(i) on which user u sent its pilot.
    yf0: [M, n_sc]; pilots: [n_sc]; returns [M, K, n_sc].
    """
    yf0 = np.asarray(yf0, dtype=np.complex128)
    p = np.asarray(pilots).astype(np.complex128)
    M, n_sc = yf0.shape
    g = pilot_groups(n_sc, K)
    with np.errstate(divide="ignore", invalid="ignore"):
        ls = yf0 * np.conj(p)[None, :] / (np.abs(p) ** 2)[None, :]
    H = np.empty((M, K, n_sc), dtype=np.complex128)
    for u in range(K):
        H[:, u, :] = ls[:, g * K + u]
    return H


# ------------------------------------------------------------------------- equal
def cholesky_lower(A):
    """Textbook Cholesky-Crout, column by column: A = L L^H, L lower with a
    real positive diagonal.  A: [..., K, K] Hermitian (only its lower triangle
    is read).  Returns (L, ok); ok is False where a pivot is <= 0 or not finite,
    and the affected entries of L are NaN."""
    A = np.asarray(A, dtype=np.complex128)
    K = A.shape[-1]
    L = np.zeros_like(A)
    ok = np.ones(A.shape[:-2], dtype=bool)
    for j in range(K):
        d = A[..., j, j].real - np.sum(np.abs(L[..., j, :j]) ** 2, axis=-1)
        good = np.isfinite(d) & (d > 0)
        ok &= good
        ljj = np.sqrt(np.where(good, d, np.nan))
        L[..., j, j] = ljj
        for i in range(j + 1, K):
            s = np.sum(L[..., i, :j] * np.conj(L[..., j, :j]), axis=-1)
            L[..., i, j] = (A[..., i, j] - s) / ljj
    return L, ok


def forward_sub(L, B):
    """Solve L W = B by forward substitution.  L [..., K, K], B [..., K, R]."""
    K = L.shape[-1]
    W = np.zeros(np.broadcast_shapes(L.shape[:-2], B.shape[:-2]) + B.shape[-2:],
                 dtype=np.complex128)
    for i in range(K):
        s = np.einsum("...k,...kr->...r", L[..., i, :i], W[..., :i, :])
        W[..., i, :] = (B[..., i, :] - s) / L[..., i, i][..., None]
    return W


def back_sub_h(L, W):
    """Solve L^H X = W by back substitution (L^H is upper triangular)."""
    K = L.shape[-1]
    X = np.zeros_like(W, dtype=np.complex128)
    for i in range(K - 1, -1, -1):
        s = np.einsum("...k,...kr->...r", np.conj(L[..., i + 1:, i]), X[..., i + 1:, :])
        X[..., i, :] = (W[..., i, :] - s) / L[..., i, i][..., None]
    return X


def _per_subcarrier(H, Y):
    Hs = np.moveaxis(np.asarray(H, dtype=np.complex128), -1, 0)   # [n_sc, M, K]
    Ys = np.moveaxis(np.asarray(Y, dtype=np.complex128), -1, 0)   # [n_sc, M, D]
    return Hs, Ys


def regularised_gram(Hs, n0: float, detector: int):
    """A = H^H H (ZF) or H^H H + N0 I (MMSE), per subcarrier."""
    Hh = np.conj(np.swapaxes(Hs, -1, -2))
    A = Hh @ Hs
    if detector == MMSE:
        A = A + n0 * np.eye(Hs.shape[-1])[None]
    return A


def detect_stage(H, Y, n0: float, detector: int = ZF, want_kappa: bool = False):
    """Linear ZF / MMSE detection of every data symbol on every subcarrier.

    H: [M, K, n_sc] channel estimate; Y: [M, D, n_sc] received data symbols.
    Per subcarrier: A = H^H H (+ N0 I); A = L L^H; z_s = H^H y_s;
    x_hat_s = A^{-1} z_s by forward then back substitution;
    d_u = [A^{-1}]_uu = sum_j |[L^{-1}]_ju|^2.
    ZF:   x_tilde = x_hat,        nu_u = N0 d_u.
    MMSE: mu_u = 1 - N0 d_u,      x_tilde_u = x_hat_u / mu_u,
          nu_u = (1 - mu_u)/mu_u  (unbiased estimate and its noise variance).
    Breakdown (a pivot <= 0, or mu <= 0) and non-finite inputs give erasures:
    x_tilde = 0, nu = +inf.
    Returns dict(xt [K, D, n_sc], nu [K, n_sc], flags [n_sc] uint8, xhat, d, mu,
    and kappa [n_sc] = exact 2-norm condition number of A if asked).
    """
    Hs, Ys = _per_subcarrier(H, Y)
    n_sc, M, K = Hs.shape
    fin = np.isfinite(Hs).all(axis=(1, 2)) & np.isfinite(Ys).all(axis=(1, 2))
    Hs = np.where(fin[:, None, None], Hs, 0.0)
    Ys = np.where(fin[:, None, None], Ys, 0.0)
    A = regularised_gram(Hs, n0, detector)
    with np.errstate(invalid="ignore", divide="ignore"):
        L, ok = cholesky_lower(A)
        Z = np.conj(np.swapaxes(Hs, -1, -2)) @ Ys
        Xh = back_sub_h(L, forward_sub(L, Z))
        Linv = forward_sub(L, np.broadcast_to(np.eye(K, dtype=np.complex128), (n_sc, K, K)))
        d = np.sum(np.abs(Linv) ** 2, axis=-2)          # [n_sc, K]
        if detector == MMSE:
            mu = 1.0 - n0 * d
            ok &= np.all(mu > 0, axis=-1)
            xt = Xh / mu[:, :, None]
            nu = (1.0 - mu) / mu
        else:
            mu = np.ones_like(d)
            xt = Xh
            nu = n0 * d
    flags = np.zeros(n_sc, dtype=np.uint8)
    flags[~ok & fin] |= FLAG_BREAKDOWN
    flags[~fin] |= FLAG_NONFINITE
    bad = flags != 0
    xt[bad] = 0.0
    nu[bad] = np.inf
    out = dict(xt=np.ascontiguousarray(np.moveaxis(xt, 0, -1)),     # [K, D, n_sc]
               nu=np.ascontiguousarray(nu.T),                        # [K, n_sc]
               flags=flags,
               xhat=np.moveaxis(Xh, 0, -1), d=d.T, mu=mu.T, ok=ok & fin)
    if want_kappa:
        ev = np.linalg.eigvalsh(np.where(bad[:, None, None], np.eye(K), A))
        with np.errstate(divide="ignore"):
            kap = ev[:, -1] / ev[:, 0]
        kap[bad] = np.inf
        out["kappa"] = kap
    return out


# ------------------------------------------------------------------------- demod
def constellation(q: int):
    """All 2^q Gray square-QAM points (unit average energy) and their labels.

    Point index c has bits b_j = (c >> (q-1-j)) & 1, b0 first.  b0, b2, b4 pick
    the in-phase level and b1, b3, b5 the quadrature level:
      QPSK  level(b)          = (1-2b)                       / sqrt(2)
      16QAM level(b, b')      = (1-2b) (2 - (1-2b'))         / sqrt(10)
      64QAM level(b, b', b'') = (1-2b) (4 - (1-2b')(2 - (1-2b''))) / sqrt(42)
    """
    n = 1 << q
    labels = np.array([[(c >> (q - 1 - j)) & 1 for j in range(q)] for c in range(n)],
                      dtype=np.int64)
    s = 1 - 2 * labels.astype(np.float64)
    if q == 2:
        re, im, scale = s[:, 0], s[:, 1], math.sqrt(2.0)
    elif q == 4:
        re = s[:, 0] * (2 - s[:, 2])
        im = s[:, 1] * (2 - s[:, 3])
        scale = math.sqrt(10.0)
    elif q == 6:
        re = s[:, 0] * (4 - s[:, 2] * (2 - s[:, 4]))
        im = s[:, 1] * (4 - s[:, 3] * (2 - s[:, 5]))
        scale = math.sqrt(42.0)
    else:
        raise ValueError("q must be 2, 4 or 6")
    return (re + 1j * im) / scale, labels


def demod_stage(xt, nu, q: int) -> np.ndarray:
    """Max-log LLR by brute force: LLR_j = (min_{c: b_j=1} |x-c|^2
    - min_{c: b_j=0} |x-c|^2) / nu, sign convention ln P(b=0)/P(b=1).

    xt: [K, D, n_sc]; nu: [K, n_sc]; returns [K, D, n_sc, q] float64.
    An erased stream (nu = +inf) gives LLR = 0.
    """
    xt = np.asarray(xt, dtype=np.complex128)
    nu = np.asarray(nu, dtype=np.float64)
    pts, lab = constellation(q)
    K = xt.shape[0]
    llr = np.empty(xt.shape + (q,), dtype=np.float64)
    for u in range(K):
        dist = np.abs(xt[u][..., None] - pts) ** 2            # [D, n_sc, 2^q]
        for j in range(q):
            d1 = dist[..., lab[:, j] == 1].min(axis=-1)
            d0 = dist[..., lab[:, j] == 0].min(axis=-1)
            with np.errstate(invalid="ignore"):
                v = (d1 - d0) / nu[u][None, :]
            llr[u, ..., j] = np.where(np.isinf(nu[u])[None, :], 0.0, v)
    return llr


# ---------------------------------------------------------------- full forward
def forward(x, pilots, shape, n0: float, detector: int = ZF, want_kappa=False):
    """One frame: time samples [M][S][cp+N] -> all stage outputs."""
    Yf = fft_stage(x, shape.n_fft, shape.n_sc, shape.cp_len)          # [M, S, n_sc]
    H = csi_stage(Yf[:, 0, :], pilots, shape.K)
    det = detect_stage(H, Yf[:, 1:, :], n0, detector, want_kappa=want_kappa)
    llr = demod_stage(det["xt"], det["nu"], shape.qam_bits)
    return dict(yf=Yf, h=H, llr=llr, **det)


def hard_bits(llr) -> np.ndarray:
    """Hard decision: bit 1 iff LLR < 0 (LLR == 0 decides 0)."""
    return (np.asarray(llr) < 0).astype(np.uint8)


# ------------------------------------------------------------------- loss + adjoint
def bce_loss(llr, bits):
    """Mean BCE-with-logits with logit(bit = 1) = -LLR; returns (loss, dloss/dLLR)."""
    z = -np.asarray(llr, dtype=np.float64)
    t = np.asarray(bits, dtype=np.float64)
    n = z.size
    loss = np.sum(np.maximum(z, 0) - z * t + np.log1p(np.exp(-np.abs(z)))) / n
    sig = 1.0 / (1.0 + np.exp(-z))
    return loss, (t - sig) / n


def demod_adjoint(xt, nu, q: int, dllr):
    """Pull dL/dLLR back to x_tilde (complex, dL/dRe + j dL/dIm) and nu.

    dLLR_j/dx = 2 (c0* - c1*) / nu with c_b* the nearest point whose bit j is b
    (ties go to the lowest point index); dLLR_j/dnu = -LLR_j / nu.
    """
    xt = np.asarray(xt, dtype=np.complex128)
    nu = np.asarray(nu, dtype=np.float64)
    pts, lab = constellation(q)
    llr = demod_stage(xt, nu, q)
    gx = np.zeros_like(xt)
    gnu = np.zeros_like(nu)
    K = xt.shape[0]
    for u in range(K):
        erased = np.isinf(nu[u])
        dist = np.abs(xt[u][..., None] - pts) ** 2
        for j in range(q):
            m1 = np.flatnonzero(lab[:, j] == 1)
            m0 = np.flatnonzero(lab[:, j] == 0)
            c1 = pts[m1][np.argmin(dist[..., m1], axis=-1)]
            c0 = pts[m0][np.argmin(dist[..., m0], axis=-1)]
            g = dllr[u, ..., j]
            with np.errstate(invalid="ignore"):
                gx[u] += np.where(erased[None, :], 0.0, g * 2.0 * (c0 - c1) / nu[u][None, :])
                gnu[u] += np.where(erased, 0.0, np.sum(g * (-llr[u, ..., j]) / nu[u][None, :], axis=0))
    return gx, gnu


def detect_adjoint(H, Y, n0: float, detector: int, gxt, gnu):
    """Pull (dL/dx_tilde, dL/dnu) back to the channel estimate and the data.

    With A = H^H H (+N0 I), x_hat_s = A^{-1} H^H y_s, r_s = y_s - H x_hat_s,
    g_hat = dL/dx_hat (MMSE: g / mu), e_u the weight of d_u = [A^{-1}]_uu:
      ZF   e_u = N0 gnu_u
      MMSE e_u = N0 (Re sum_s conj(g_su) x_hat_su / mu_u^2 + gnu_u / mu_u^2)
    and V = A^{-1} G_hat, the gradients are
      dL/dY = H V
      dL/dH = Y V^H - H (X_hat V^H + V X_hat^H + 2 A^{-1} diag(e) A^{-1}).
    Erased subcarriers pass no gradient.
    H: [M, K, n_sc], Y: [M, D, n_sc], gxt: [K, D, n_sc], gnu: [K, n_sc].
    Returns (gH [M, K, n_sc], gY [M, D, n_sc]).
    """
    Hs, Ys = _per_subcarrier(H, Y)
    n_sc, M, K = Hs.shape
    det = detect_stage(H, Y, n0, detector)
    ok = det["ok"]
    okk = ok[:, None, None]
    # erased subcarriers are replaced by a harmless stand-in and zeroed at the end
    Hs = np.where(okk, Hs, np.eye(M, K)[None])
    Ys = np.where(okk, Ys, 0.0)
    A = regularised_gram(Hs, n0, detector)
    L, _ = cholesky_lower(A)
    Xh = np.where(okk, np.moveaxis(det["xhat"], -1, 0), 0.0)        # [n_sc, K, D]
    G = np.where(okk, np.moveaxis(np.asarray(gxt, dtype=np.complex128), -1, 0), 0.0)
    gn = np.where(ok[:, None], np.asarray(gnu, dtype=np.float64).T, 0.0)   # [n_sc, K]
    if detector == MMSE:
        mu = np.where(ok[:, None], det["mu"].T, 0.5)
        Gh = G / mu[:, :, None]
        c = np.real(np.sum(np.conj(G) * Xh, axis=-1)) / mu ** 2
        e = n0 * (c + gn / mu ** 2)
    else:
        Gh = G
        e = n0 * gn
    V = back_sub_h(L, forward_sub(L, Gh))
    Linv = forward_sub(L, np.broadcast_to(np.eye(K, dtype=np.complex128), (n_sc, K, K)))
    Ainv = np.conj(np.swapaxes(Linv, -1, -2)) @ Linv
    Vh = np.conj(np.swapaxes(V, -1, -2))
    C = Xh @ Vh + V @ np.conj(np.swapaxes(Xh, -1, -2)) + 2.0 * (Ainv * e[:, None, :]) @ Ainv
    gH = Ys @ Vh - Hs @ C
    gY = Hs @ V
    gH[~ok] = 0.0
    gY[~ok] = 0.0
    return np.ascontiguousarray(np.moveaxis(gH, 0, -1)), np.ascontiguousarray(np.moveaxis(gY, 0, -1))


def csi_adjoint(gH, pilots, n_sc: int):
    """dL/dYf0[m][q] = p[q]/|p[q]|^2 * sum_{i in group g} dL/dH[m][u][i] for
    q = g K + u; pilot subcarriers past the last full group get 0, and so do
    zero pilots (their estimates are non-finite and erased downstream)."""
    gH = np.asarray(gH, dtype=np.complex128)
    M, K, _ = gH.shape
    p = np.asarray(pilots).astype(np.complex128)
    g = pilot_groups(n_sc, K)
    G = n_sc // K
    out = np.zeros((M, n_sc), dtype=np.complex128)
    for u in range(K):
        acc = np.zeros((M, G), dtype=np.complex128)
        np.add.at(acc.T, g, gH[:, u, :].T)
        q = np.arange(G) * K + u
        pp = np.abs(p[q]) ** 2
        scale = np.where(pp > 0, p[q] / np.where(pp > 0, pp, 1.0), 0.0)
        out[:, q] = acc * scale[None, :]
    return out


def fft_adjoint(gYf, n_fft: int, n_sc: int, cp_len: int = 0):
    """dL/dx[cp+n] = sum_i dL/dYf[i] exp(+j 2 pi bin(i) n / N); CP samples get 0."""
    gYf = np.asarray(gYf, dtype=np.complex128)
    grid = np.zeros(gYf.shape[:-1] + (n_fft,), dtype=np.complex128)
    grid[..., used_bins(n_fft, n_sc)] = gYf
    seg = np.fft.ifft(grid, axis=-1) * n_fft
    out = np.zeros(gYf.shape[:-1] + (cp_len + n_fft,), dtype=np.complex128)
    out[..., cp_len:] = seg
    return out


def backward(x, pilots, shape, n0: float, detector: int, dllr):
    """Adjoint of the whole forward map: dL/dLLR -> (dL/dx, dL/dH)."""
    fw = forward(x, pilots, shape, n0, detector)
    gxt, gnu = demod_adjoint(fw["xt"], fw["nu"], shape.qam_bits, dllr)
    gH, gY = detect_adjoint(fw["h"], fw["yf"][:, 1:, :], n0, detector, gxt, gnu)
    gYf = np.zeros_like(fw["yf"])
    gYf[:, 1:, :] = gY
    gYf[:, 0, :] = csi_adjoint(gH, pilots, shape.n_sc)
    gx = fft_adjoint(gYf, shape.n_fft, shape.n_sc, shape.cp_len)
    return gx, gH


# --------------------------------------------------- cascaded-channel phase grad
def cascaded_theta_grad(gx, shape, theta, Gm, Fm, amp, symbols, pilots):
    """dL/dtheta for x synthesised from H = (1/sqrt(n_el)) G diag(e^{j theta}) F
    + 0.1 H_d (frequency flat), given gx = dL/dx (complex convention).

    x = ifft(grid) (+ CP copy) is linear in the grid; the grid is
    Y[m][s][i] = sum_u amp_u H[m][u] s_u[s][i] (pilot symbol: only the comb
    owner of subcarrier i).  Pull-backs: grid <- fft(gx)/N, H <- amp_u *
    sum conj(s) gY, theta_k <- Re sum conj(gH) (j/sqrt(n_el)) G[:,k] e^{j theta_k} F[k,:].
    """
    M, K, N, n_sc, cp = shape.M, shape.K, shape.n_fft, shape.n_sc, shape.cp_len
    gx = np.asarray(gx, dtype=np.complex128)
    seg = gx[..., cp:].copy()
    if cp:
        seg[..., N - cp:] += gx[..., :cp]
    ggrid = np.fft.fft(seg, axis=-1) / N
    gY = ggrid[..., used_bins(N, n_sc)]                      # [M, S, n_sc]
    pu = np.arange(n_sc) % K
    gHe = np.einsum("mdi,udi->mu", gY[:, 1:, :], np.conj(symbols))
    for u in range(K):
        sel = pu == u
        gHe[:, u] += gY[:, 0, sel] @ np.conj(np.asarray(pilots, dtype=np.complex128)[sel])
    gH = gHe * np.asarray(amp)[None, :]
    n_el = Gm.shape[1]
    ej = np.exp(1j * np.asarray(theta))
    # dH[m][u]/dtheta_k = (j/sqrt(n_el)) G[m][k] e^{j theta_k} F[k][u]
    t = np.einsum("mu,mk,ku->k", np.conj(gH), Gm, Fm)
    return np.real(t * 1j * ej) / math.sqrt(n_el)


# ---------------------------------------------------------------------- downlink
# The transmit direction beside the uplink path (the `modul`, `precode` and
# `ifft` macros of the paper's preamble): QAM mapping,
# a zero-forcing precoder built from the same Gram matrix and Cholesky factor
# as the detector, and the inverse transform with a cyclic prefix.
def modulate_stage(bits, q: int) -> np.ndarray:
    """bits [..., q] (b0 first) -> the Gray square-QAM point with that label,
    i.e. constellation(q)'s point index c = sum_j b_j 2^(q-1-j)."""
    pts, _ = constellation(q)
    b = np.asarray(bits).astype(np.int64)
    if b.shape[-1] != q:
        raise ValueError("last axis must hold the q bits")
    idx = np.zeros(b.shape[:-1], dtype=np.int64)
    for j in range(q):
        idx = idx * 2 + b[..., j]
    return pts[idx]


def precode_stage(H, S, n0: float = 1.0, detector: int = ZF):
    """Zero-forcing precoding with the uplink estimate (reciprocity): per
    subcarrier X = H A^{-1} S with A = H^H H (ZF) or H^H H + N0 I (the
    regularised form, detector = MMSE), so that a downlink channel H^H gives
    H^H X = S for ZF.  A^{-1} S by the same Cholesky and two triangular solves
    as detect_stage; no power normalisation.  A breakdown (pivot <= 0) or a
    non-finite channel value transmits nothing on that subcarrier (X = 0) and
    flags it.

    H: [M, K, n_sc]; S: [K, D, n_sc]; returns dict(x [M, D, n_sc], flags [n_sc])."""
    Hs = np.moveaxis(np.asarray(H, dtype=np.complex128), -1, 0)     # [n_sc, M, K]
    Ss = np.moveaxis(np.asarray(S, dtype=np.complex128), -1, 0)     # [n_sc, K, D]
    fin = np.isfinite(Hs).all(axis=(1, 2))
    Hs = np.where(fin[:, None, None], Hs, 0.0)
    A = regularised_gram(Hs, n0, detector)
    with np.errstate(invalid="ignore", divide="ignore"):
        L, ok = cholesky_lower(A)
        W = back_sub_h(L, forward_sub(L, Ss))                         # A^{-1} S
        X = Hs @ W                                                    # [n_sc, M, D]
    flags = np.zeros(Hs.shape[0], dtype=np.uint8)
    flags[~ok & fin] |= FLAG_BREAKDOWN
    flags[~fin] |= FLAG_NONFINITE
    X[flags != 0] = 0.0
    return dict(x=np.ascontiguousarray(np.moveaxis(X, 0, -1)), flags=flags)


def ifft_stage(Xf, n_fft: int, n_sc: int, cp_len: int = 0) -> np.ndarray:
    """Inverse of fft_stage's used-bin transform, unscaled, with a cyclic
    prefix: x[n] = sum_i Xf[i] exp(+j 2 pi bin(i) n / N) for n = 0..N-1, then
    the last cp_len samples are prepended (so fft_stage(ifft_stage(X)) = N X).

    Xf: [..., n_sc]; returns [..., cp_len + n_fft] complex128."""
    Xf = np.asarray(Xf, dtype=np.complex128)
    grid = np.zeros(Xf.shape[:-1] + (n_fft,), dtype=np.complex128)
    grid[..., used_bins(n_fft, n_sc)] = Xf
    seg = np.fft.ifft(grid, axis=-1) * n_fft
    return np.concatenate([seg[..., n_fft - cp_len:], seg], axis=-1)


# ---------------------------------------------------------- pins: brute-force ML
def ml_maxlog(Hs, y, n0: float, q: int):
    """Joint max-log ML LLRs by enumeration of every K-user symbol vector.

    Hs: [M, K] channel, y: [M] received; metric |y - H x|^2 / N0.
    Returns [K, q].  Exponential in K*q: pins only.
    """
    pts, lab = constellation(q)
    M, K = Hs.shape
    n = len(pts)
    idx = np.array(np.meshgrid(*([np.arange(n)] * K), indexing="ij")).reshape(K, -1).T
    X = pts[idx]                                         # [n^K, K]
    metric = np.sum(np.abs(y[None, :] - X @ Hs.T) ** 2, axis=-1) / n0
    out = np.empty((K, q))
    for u in range(K):
        for j in range(q):
            b = lab[idx[:, u], j]
            out[u, j] = metric[b == 1].min() - metric[b == 0].min()
    return out
