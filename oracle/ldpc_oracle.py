"""Plain FP64 oracle of layered decoding of quasi-cyclic LDPC codes.

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Slow on purpose;
each step can be checked against its definition by eye.

The paper names the channel-decoding stage (the `dec` macro of its preamble,
beside `enc`) and the LDPC notation it would use (lifting size Z_c, the
lifting-size set, code-block size K_cb, filler bits, code rate R) but defines
no decoder.  What is computed here is the textbook one:

  code        a quasi-cyclic parity-check matrix given by a base matrix B
              (mb x nb): entry -1 is a Z x Z zero block, entry s in [0, Z)
              the identity with its columns cyclically shifted by s, i.e.
              row r of the block has its one in column (r + s) mod Z.
              Codeword length N = nb Z; check (i Z + r) involves bit
              j Z + (r + B[i][j]) mod Z of every block column j with
              B[i][j] >= 0.
  LLRs        ln P(bit = 0) / P(bit = 1), the receiver's convention; the hard
              decision is bit 1 iff the LLR is < 0 (0 decides bit 0).
  schedule    layered belief propagation: one layer per block row, in order
              0 .. mb-1; within a layer the Z checks touch disjoint bits, so
              their order does not matter.  For check c and each of its bits
              v (block columns in increasing order): Q_cv = L_v - R_cv,
              new R_cv from the check rule on {Q_cv'}, L_v = Q_cv + R_cv.
              L starts at the channel LLRs, every R at 0.
  check rule  normalised min-sum: R_cv = alpha * prod_{v' != v} sgn(Q_cv')
              * min_{v' != v} |Q_cv'|, sgn(0) = +1; or the sum-product rule
              R_cv = 2 atanh(prod_{v' != v} tanh(Q_cv' / 2)) (pins only).
  stopping    the syndrome H c of the hard decisions is checked before the
              first iteration and after every iteration (all layers); the
              decoder stops at the first zero syndrome.  The iteration count
              returned is the number of full iterations run (0 when the
              channel word is already a codeword).

Arithmetic: float64 by default.  With dtype=np.float32 every operation is
rounded to FP32 as it is made (Q = L - R, alpha * min, L = Q + R; the signs
and minima are exact): the precision in which the FP32 decoder takes its
decisions (signs, argmins, hard bits, the stopping test), so that the two can
be compared bit for bit.  The expanded H is built entry by entry.
"""
from __future__ import annotations

import math

import numpy as np


def expand(base, z: int) -> np.ndarray:
    """The parity-check matrix H (uint8, [mb z][nb z]) of base matrix `base`."""
    base = np.asarray(base)
    mb, nb = base.shape
    H = np.zeros((mb * z, nb * z), dtype=np.uint8)
    for i in range(mb):
        for j in range(nb):
            s = int(base[i, j])
            if s < 0:
                continue
            for r in range(z):
                H[i * z + r, j * z + (r + s) % z] = 1
    return H


def syndrome(H, bits) -> np.ndarray:
    """H c over GF(2)."""
    return (np.asarray(H, dtype=np.int64) @ np.asarray(bits, dtype=np.int64)) % 2


def hard(llr) -> np.ndarray:
    return (np.asarray(llr) < 0).astype(np.uint8)


def _sgn(x: float) -> float:
    return -1.0 if x < 0 else 1.0


def check_minsum(q, alpha: float, dtype=np.float64) -> np.ndarray:
    """Normalised min-sum messages of one check from its incoming Q values,
    each excluding its own edge (the definition, O(d^2)): the sign product
    times the rounded product alpha * min."""
    d = len(q)
    out = np.zeros(d, dtype=dtype)
    a = dtype(alpha)
    for k in range(d):
        s, m = 1.0, None
        for kk in range(d):
            if kk == k:
                continue
            s *= _sgn(q[kk])
            m = abs(q[kk]) if m is None else min(m, abs(q[kk]))
        out[k] = dtype(s) * dtype(a * dtype(m))
    return out


def check_sumproduct(q) -> np.ndarray:
    """Sum-product (tanh rule) messages of one check, each excluding its own edge."""
    d = len(q)
    out = np.zeros(d)
    for k in range(d):
        p = 1.0
        for kk in range(d):
            if kk != k:
                p *= math.tanh(q[kk] / 2.0)
        p = min(max(p, -1.0 + 1e-15), 1.0 - 1e-15)
        out[k] = 2.0 * math.atanh(p)
    return out


def layer_edges(base, z: int, i: int, r: int):
    """Bits of check (i z + r): one per non-zero block of row i, block columns
    in increasing order."""
    base = np.asarray(base)
    return [(j, j * z + (r + int(base[i, j])) % z) for j in range(base.shape[1]) if base[i, j] >= 0]


def syndrome_qc(base, z: int, bits) -> np.ndarray:
    """H c over GF(2) from the base matrix, without expanding H: check i z + r
    is the XOR of bit j z + (r + B[i][j]) mod z over the row's blocks."""
    base = np.asarray(base)
    bits = np.asarray(bits, dtype=np.uint8)
    r = np.arange(z)
    out = np.zeros(base.shape[0] * z, dtype=np.uint8)
    for i in range(base.shape[0]):
        acc = np.zeros(z, dtype=np.uint8)
        for j in range(base.shape[1]):
            if base[i, j] >= 0:
                acc ^= bits[j * z + (r + int(base[i, j])) % z]
        out[i * z:(i + 1) * z] = acc
    return out


def _layer_minsum(q, alpha, dtype):
    """check_minsum applied to the z checks of a layer at once: q is [d][z]
    (row k = the k-th bit of every check); the same per-check definition."""
    d = q.shape[0]
    a = dtype(alpha)
    sg = np.where(q < 0, dtype(-1.0), dtype(1.0))
    out = np.zeros_like(q)
    for k in range(d):
        others = [kk for kk in range(d) if kk != k]
        s = np.prod(sg[others], axis=0)
        m = np.min(np.abs(q[others]), axis=0)
        out[k] = s * (a * m)
    return out


def _layer_sumproduct(q):
    d = q.shape[0]
    t = np.tanh(q / 2.0)
    out = np.zeros_like(q)
    for k in range(d):
        p = np.prod(t[[kk for kk in range(d) if kk != k]], axis=0)
        out[k] = 2.0 * np.arctanh(np.clip(p, -1.0 + 1e-15, 1.0 - 1e-15))
    return out


def decode(base, z: int, llr, max_iter: int, alpha: float = 0.75, rule: str = "minsum",
           early_stop: bool = True, dtype=np.float64):
    """Layered decoding of one codeword.  Returns (posterior LLRs, hard bits,
    iterations run).  The z checks of a layer touch disjoint bits, so they are
    updated together (numpy over the check index r)."""
    base = np.asarray(base)
    mb, nb = base.shape
    L = np.asarray(llr).astype(dtype)
    if L.shape != (nb * z,):
        raise ValueError("llr must have nb * z entries")
    for i in range(mb):
        if np.sum(base[i] >= 0) < 2:
            raise ValueError("every block row needs two or more non-zero blocks")
    r = np.arange(z)
    layers = []                                # per layer: block columns and their bit index arrays
    for i in range(mb):
        cols = [j for j in range(nb) if base[i, j] >= 0]
        layers.append((cols, np.stack([j * z + (r + int(base[i, j])) % z for j in cols])))
    R = [np.zeros((len(cols), z), dtype=dtype) for cols, _ in layers]
    if early_stop and not np.any(syndrome_qc(base, z, hard(L))):
        return L, hard(L), 0
    for it in range(1, max_iter + 1):
        for i, (cols, v) in enumerate(layers):
            q = (L[v] - R[i]).astype(dtype)
            rn = _layer_minsum(q, alpha, dtype) if rule == "minsum" else _layer_sumproduct(q)
            L[v] = (q + rn).astype(dtype)
            R[i] = rn
        if early_stop and not np.any(syndrome_qc(base, z, hard(L))):
            return L, hard(L), it
    return L, hard(L), max_iter


def decode_batch(base, z: int, llr, max_iter: int, alpha: float = 0.75, dtype=np.float64):
    """decode() of each row of llr [n_cw][nb z]: (posteriors, bits, iterations)."""
    outs = [decode(base, z, row, max_iter, alpha, dtype=dtype) for row in np.asarray(llr)]
    return (np.stack([o[0] for o in outs]), np.stack([o[1] for o in outs]),
            np.array([o[2] for o in outs], dtype=np.int32))


def map_llrs_by_enumeration(H, llr) -> np.ndarray:
    """Exact bitwise MAP LLRs by enumerating every codeword of H (tiny codes):
    P(c | y) is proportional to exp(sum_v (1 - 2 c_v) llr_v / 2)."""
    H = np.asarray(H, dtype=np.int64)
    n = H.shape[1]
    llr = np.asarray(llr, dtype=np.float64)
    num = np.full(n, -math.inf)                 # log-sum over codewords with c_v = 0
    den = np.full(n, -math.inf)                 # ... with c_v = 1
    for word in range(1 << n):
        c = np.array([(word >> v) & 1 for v in range(n)], dtype=np.int64)
        if np.any((H @ c) % 2):
            continue
        metric = float(np.sum((1 - 2 * c) * llr) / 2.0)
        for v in range(n):
            if c[v] == 0:
                num[v] = np.logaddexp(num[v], metric)
            else:
                den[v] = np.logaddexp(den[v], metric)
    return num - den
