"""Differentiable (torch) synthesis of a cascaded-channel frame as a function of
the element phases theta, for gradients dL/dtheta by autograd.

Same construction as ``synth.frames`` for the cascaded model: H = G
diag(exp(j theta)) F / sqrt(n_el) + 0.1 H_d (frequency flat), user power
folded in, comb pilots in symbol 0, data in symbols 1..D, numpy-style ifft,
the frame's own fixed time-domain noise, complex64 output.
"""
import math

import numpy as np
import torch

from .frames import pilot_user, used_bins


def cascaded_x(theta, frame, device="cuda"):
    """x [1][M][S][cp+N] complex64 on `device`, differentiable in theta
    (a float64 tensor of the frame's element count)."""
    ex = frame.extra
    sh = frame.shape
    M, K, N, n_sc, S, cp = sh.M, sh.K, sh.n_fft, sh.n_sc, sh.n_sym, sh.cp_len
    c128 = torch.complex128
    Gm = torch.as_tensor(ex["G"], dtype=c128, device=device)
    Fm = torch.as_tensor(ex["F"], dtype=c128, device=device)
    Hd = torch.as_tensor(ex["Hd"], dtype=c128, device=device)
    amp = torch.as_tensor(ex["amp"], dtype=torch.float64, device=device)
    n_el = Gm.shape[1]
    ej = torch.polar(torch.ones_like(theta), theta)
    H = (Gm * ej[None, :]) @ Fm / math.sqrt(n_el) + 0.1 * Hd         # [M][K]
    He = H * amp[None, :]
    sym = torch.as_tensor(frame.symbols, dtype=c128, device=device)     # [K][D][n_sc]
    pil = torch.as_tensor(frame.pilots.astype(np.complex128), device=device)
    pu = torch.as_tensor(pilot_user(n_sc, K), device=device)
    y0 = He[:, pu] * pil[None, :]                                        # [M][n_sc]
    yd = torch.einsum("mu,udi->mdi", He, sym)                            # [M][D][n_sc]
    Y = torch.cat([y0[:, None, :], yd], dim=1)                           # [M][S][n_sc]
    grid = torch.zeros((M, S, N), dtype=c128, device=device)
    grid[..., torch.as_tensor(used_bins(N, n_sc), device=device)] = Y
    x = torch.fft.ifft(grid, dim=-1) + torch.as_tensor(ex["noise_t"], dtype=c128, device=device)
    if cp:
        x = torch.cat([x[..., N - cp:], x], dim=-1)
    return x.to(torch.complex64)[None]
