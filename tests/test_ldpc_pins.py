"""CPU pins of the LDPC oracle (layered normalised min-sum over quasi-cyclic
codes) against what the mathematics fixes: the circulant expansion against
shifted identities built by numpy, the generator's codewords, closed forms of
one parity check and of a repetition code, exact MAP decoding by enumeration
on a cycle-free graph, and decoding of noisy codewords."""
import math

import numpy as np
import pytest

from oracle import ldpc_oracle as L
from synth import ldpc as G


def test_expand_matches_shifted_identities():
    rng = np.random.default_rng(1)
    z = 7
    base = rng.integers(-1, z, (3, 5)).astype(np.int16)
    H = L.expand(base, z)
    for i in range(3):
        for j in range(5):
            blk = H[i * z:(i + 1) * z, j * z:(j + 1) * z]
            want = np.zeros((z, z)) if base[i, j] < 0 else np.roll(np.eye(z), int(base[i, j]), axis=1)
            assert np.array_equal(blk, want)
    # row r of a block with shift s has its one in column (r + s) mod z
    assert H[2, 0 * z + (2 + base[0, 0]) % z] == 1 or base[0, 0] < 0


def test_generator_codewords_satisfy_the_checks():
    base = G.random_base(5, 7, 16, 3, seed=2)
    H = L.expand(base, 16)
    cw = G.make_codewords(base, 16, 6, seed=3)
    assert cw.shape == (6, 12 * 16)
    for c in cw:
        assert not np.any(L.syndrome(H, c))
    # the staircase: every information column is used, the parity part is lower bidiagonal
    assert np.all(np.sum(base[:, :7] >= 0, axis=0) >= 3)
    par = base[:, 7:]
    assert np.all(np.diag(par) == 0) and np.all(np.diag(par, -1) == 0)
    assert np.sum(par >= 0) == 5 + 4


def test_valid_codeword_comes_back_unchanged():
    """A channel word that is already a codeword stops before the first
    iteration; without the stop, min-sum only grows the LLRs' magnitudes
    (every check's other signs agree with each bit's own)."""
    z = 16
    base = G.random_base(4, 8, z, 3, seed=4)
    c = G.make_codewords(base, z, 1, seed=5)[0]
    rng = np.random.default_rng(6)
    llr = (1.0 - 2.0 * c) * rng.uniform(0.5, 4.0, c.size)
    post, bits, it = L.decode(base, z, llr, 10)
    assert it == 0 and np.array_equal(post, llr) and np.array_equal(bits, c)
    post, bits, it = L.decode(base, z, llr, 3, early_stop=False)
    assert it == 3 and np.array_equal(bits, c)
    assert np.all(np.abs(post) >= np.abs(llr) - 1e-12)


@pytest.mark.parametrize("alpha", [1.0, 0.75])
def test_single_parity_check_one_iteration_closed_form(alpha):
    """One check over d bits (z = 1): after one iteration
    L_k = l_k + alpha * (product of the other signs) * (smallest other |l|),
    i.e. the smallest |l| for every bit but the smallest one, which gets the
    second smallest."""
    rng = np.random.default_rng(7)
    d = 9
    lam = rng.standard_normal(d) * 3
    post, _, _ = L.decode(np.zeros((1, d), np.int16), 1, lam, 1, alpha, early_stop=False)
    order = np.argsort(np.abs(lam))
    m1, m2 = abs(lam[order[0]]), abs(lam[order[1]])
    total_sign = np.prod(np.where(lam < 0, -1.0, 1.0))
    for k in range(d):
        own = -1.0 if lam[k] < 0 else 1.0
        mag = m2 if k == order[0] else m1
        assert post[k] == pytest.approx(lam[k] + alpha * total_sign * own * mag, abs=1e-12)


@pytest.mark.parametrize("rule", ["minsum", "sumproduct"])
def test_repetition_chain_converges_to_the_sum(rule):
    """Checks c_k + c_{k+1} = 0 make a repetition code (a chain, cycle-free):
    its exact bitwise MAP LLR is the sum of all channel LLRs.  Degree-2 checks
    pass the other bit's Q unchanged under both rules (alpha = 1), and the
    layered schedule reaches the sum within n iterations."""
    n = 8
    base = np.full((n - 1, n), -1, np.int16)
    for k in range(n - 1):
        base[k, k] = base[k, k + 1] = 0
    lam = np.random.default_rng(8).standard_normal(n) * 2
    if rule == "minsum":
        post, _, _ = L.decode(base, 1, lam, n + 2, 1.0, early_stop=False)
    else:
        post, _, _ = L.decode(base, 1, lam, n + 2, rule="sumproduct", early_stop=False)
    assert np.allclose(post, np.sum(lam), atol=1e-9)


def test_sum_product_equals_map_on_a_tree():
    """On a cycle-free Tanner graph belief propagation is exact: the layered
    sum-product posteriors equal the bitwise MAP LLRs found by enumerating
    every codeword."""
    checks = [(0, 1, 2), (2, 3, 4), (4, 5, 6), (1, 7), (6, 8)]
    n = 9
    base = np.full((len(checks), n), -1, np.int16)
    for i, ch in enumerate(checks):
        base[i, list(ch)] = 0
    H = L.expand(base, 1)
    lam = np.random.default_rng(9).standard_normal(n) * 1.5
    post, _, _ = L.decode(base, 1, lam, 30, rule="sumproduct", early_stop=False)
    ref = L.map_llrs_by_enumeration(H, lam)
    assert np.allclose(post, ref, atol=1e-9)
    # min-sum is not exact there: it differs from MAP by more than rounding
    ms, _, _ = L.decode(base, 1, lam, 30, 1.0, early_stop=False)
    assert np.max(np.abs(ms - ref)) > 1e-3


def test_min_sum_decodes_noisy_codewords_and_stops_at_the_first_zero_syndrome():
    z = 32
    base = G.random_base(6, 6, z, 3, seed=10)        # rate 1/2, N = 384
    H = L.expand(base, z)
    cw = G.make_codewords(base, z, 6, seed=11)
    llr = G.bpsk_awgn_llrs(cw, 6.0, seed=12)
    raw = np.sum(L.hard(llr) != cw)
    assert raw > 0                                     # the channel made errors
    post, bits, its = L.decode_batch(base, z, llr, 30)
    assert np.array_equal(bits, cw)
    assert np.all(its >= 1) and np.all(its < 30)
    k = int(np.argmax(its))
    if its[k] > 1:
        p1, b1, i1 = L.decode(base, z, llr[k], int(its[k]) - 1)
        assert i1 == its[k] - 1 and np.any(L.syndrome(H, b1))
    p2, _, i2 = L.decode(base, z, llr[k], int(its[k]), early_stop=False)
    assert i2 == its[k] and np.array_equal(p2, post[k])


def test_minsum_check_rule_against_the_two_smallest():
    """The check rule excluding each edge equals the reformulation through the
    smallest and second-smallest |Q| and the total sign (the form a decoder
    stores)."""
    rng = np.random.default_rng(13)
    for d in (2, 3, 7, 19):
        q = rng.standard_normal(d) * 4
        q[rng.integers(d)] = 0.0 if d > 2 else q[0]
        got = L.check_minsum(q, 0.8)
        a = np.abs(q)
        i1 = int(np.argmin(a))
        m2 = np.min(np.delete(a, i1))
        sg = np.where(q < 0, -1.0, 1.0)
        want = 0.8 * np.prod(sg) * sg * np.where(np.arange(d) == i1, m2, a[i1])
        assert np.allclose(got, want, atol=0)


def test_fp32_mode_rounds_each_operation():
    """The FP32 mode (the precision the GPU decoder decides in) agrees with the
    FP64 decoder to FP32 rounding on a noisy word, returns float32 values, and
    rounds alpha * min once: on one check its messages are exactly
    float32(float32(alpha) * float32(min))."""
    q = np.array([0.3, -1.7, 2.25], dtype=np.float32)
    out = L.check_minsum(q, 0.75, np.float32)
    assert out.dtype == np.float32
    a = np.float32(0.75)
    assert out[0] == -(a * np.float32(1.7)) and out[1] == a * np.float32(0.3) and out[2] == -(a * np.float32(0.3))
    z = 16
    base = G.random_base(4, 4, z, 3, seed=14)
    cw = G.make_codewords(base, z, 1, seed=15)
    llr = G.bpsk_awgn_llrs(cw, 4.0, seed=16)[0]
    p64, b64, i64 = L.decode(base, z, llr, 8)
    p32, b32, i32 = L.decode(base, z, llr, 8, dtype=np.float32)
    assert p32.dtype == np.float32 and i32 == i64 and np.array_equal(b32, b64)
    assert np.max(np.abs(p32 - p64) / np.maximum(np.abs(p64), 1.0)) < 1e-5


def test_layer_form_equals_the_per_check_definition_and_sparse_syndrome():
    """The decoder's layer-at-once evaluation gives each check exactly the
    per-check definition (check_minsum, rounded the same way), and the sparse
    syndrome equals H c with H expanded entry by entry."""
    rng = np.random.default_rng(17)
    z = 12
    base = G.random_base(3, 5, z, 3, seed=18)
    H = L.expand(base, z)
    for _ in range(3):
        b = rng.integers(0, 2, 8 * z).astype(np.uint8)
        assert np.array_equal(L.syndrome_qc(base, z, b), L.syndrome(H, b))
    for dt in (np.float64, np.float32):
        q = (rng.standard_normal((5, z)) * 3).astype(dt)
        lay = L._layer_minsum(q, 0.75, dt)
        for rr in range(z):
            assert np.array_equal(lay[:, rr], L.check_minsum(q[:, rr], 0.75, dt))
