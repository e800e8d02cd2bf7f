"""Seeded quasi-cyclic LDPC codes, codewords and channel LLRs.

The transmitter side of the decoder's inputs: a random base matrix whose
parity part is a staircase (so that encoding is a running sum), the
systematic encoder of that structure, and BPSK over AWGN giving LLRs in the
receiver's convention (ln P(0) / P(1)).  Nothing here decodes: no check
update, no message passing, no syndrome test.
"""
from __future__ import annotations

import numpy as np


def random_base(mb: int, kb: int, z: int, row_weight: int, seed) -> np.ndarray:
    """Base matrix [mb][kb + mb] (int16; -1 = zero block, else a shift in
    [0, z)).  Information part: row_weight non-zero blocks per row at random
    columns with random shifts, then blocks added until every information
    column has weight 3 or more (a weight-2 column can pair with a staircase
    column into a weight-2 codeword).
    Parity part: the staircase (shift 0 on the diagonal and below it), so
    parity block i = parity block i-1 + row i's information sum."""
    rng = np.random.default_rng(seed)
    base = np.full((mb, kb + mb), -1, dtype=np.int16)
    row_weight = min(row_weight, kb)
    for i in range(mb):
        cols = rng.choice(kb, row_weight, replace=False)
        base[i, cols] = rng.integers(0, z, row_weight)
    for j in range(kb):                              # information columns of weight >= 3
        while np.sum(base[:, j] >= 0) < min(3, mb):
            free = np.flatnonzero(base[:, j] < 0)
            base[rng.choice(free), j] = rng.integers(0, z)
    for i in range(mb):
        base[i, kb + i] = 0
        if i > 0:
            base[i, kb + i - 1] = 0
    return base


def encode(base, z: int, info) -> np.ndarray:
    """Systematic codeword [info | parity] of a staircase base matrix (uint8).
    Block row i reads sum_j P^{s_ij} u_j + p_{i-1} + p_i = 0 over GF(2), where
    (P^s u)[r] = u[(r + s) mod z]."""
    base = np.asarray(base)
    mb, nb = base.shape
    kb = nb - mb
    u = np.asarray(info, dtype=np.uint8).reshape(kb, z)
    p = np.zeros((mb, z), dtype=np.uint8)
    r = np.arange(z)
    for i in range(mb):
        acc = np.zeros(z, dtype=np.uint8)
        for j in range(kb):
            s = int(base[i, j])
            if s >= 0:
                acc ^= u[j, (r + s) % z]
        if i > 0:
            acc ^= p[i - 1]
        p[i] = acc
    return np.concatenate([u.reshape(-1), p.reshape(-1)])


def bpsk_awgn_llrs(codewords, snr_db: float, seed) -> np.ndarray:
    """BPSK (bit b -> 1 - 2b) over real AWGN of variance sigma^2 = 10^(-snr/10):
    LLR = 2 y / sigma^2, float32 [n_cw][N]."""
    rng = np.random.default_rng(seed)
    c = np.asarray(codewords, dtype=np.float64)
    sigma2 = 10.0 ** (-snr_db / 10.0)
    y = (1.0 - 2.0 * c) + rng.standard_normal(c.shape) * np.sqrt(sigma2)
    return (2.0 * y / sigma2).astype(np.float32)


def make_codewords(base, z: int, n_cw: int, seed) -> np.ndarray:
    """n_cw codewords of random information bits (uint8 [n_cw][nb z])."""
    base = np.asarray(base)
    kb = base.shape[1] - base.shape[0]
    rng = np.random.default_rng(seed)
    return np.stack([encode(base, z, rng.integers(0, 2, kb * z)) for _ in range(n_cw)])
