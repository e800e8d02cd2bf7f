"""GPU layered min-sum LDPC decoder (rxphy_ldpc_decode) against the oracle in
its FP32 mode, which rounds every operation as the kernel does and so takes
the same decisions (signs, argmins, hard bits, the stopping test): posterior
LLRs, hard bits and iteration counts are compared bit for bit, on seeded
random quasi-cyclic codes (staircase parity part) with BPSK-over-AWGN LLRs.
The FP64 oracle is reported beside it.  Parity against the 3GPP base graphs
is unpinned: their tables are not available here."""
import numpy as np
import pytest

from oracle import ldpc_oracle as L
from synth import ldpc as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-ldpc]", *a, flush=True)


CASES = [
    # mb, kb, z, row weight, n_cw, snr dB, max_iter, alpha
    (4, 4, 16, 3, 6, 3.0, 12, 0.75),
    (6, 6, 32, 3, 5, 2.5, 20, 0.75),
    (5, 11, 24, 5, 4, 3.5, 15, 1.0),           # z not a multiple of 16, plain min-sum
    (8, 16, 60, 6, 3, 3.0, 10, 0.8),           # a ragged wave: 60 rows per layer
    (3, 5, 130, 4, 2, 2.0, 8, 0.75),           # z > 128: three waves per layer
]


@pytest.mark.parametrize("mb,kb,z,rw,n_cw,snr,max_iter,alpha", CASES)
def test_ldpc_decode_bitexact_against_fp32_oracle(rx, mb, kb, z, rw, n_cw, snr, max_iter, alpha):
    seed = mb * 1000 + z
    base = G.random_base(mb, kb, z, rw, seed=seed)
    cw = G.make_codewords(base, z, n_cw, seed=seed + 1)
    llr = G.bpsk_awgn_llrs(cw, snr, seed=seed + 2)
    code = rx.LdpcCode(base, z)
    post, bits, its = rx.ldpc_decode(code, torch.from_numpy(llr).cuda(), max_iter, alpha)
    post, bits, its = post.cpu().numpy(), bits.cpu().numpy(), its.cpu().numpy()
    rp, rb, ri = L.decode_batch(base, z, llr, max_iter, alpha, dtype=np.float32)
    r64, b64, i64 = L.decode_batch(base, z, llr, max_iter, alpha)
    say("code", (mb, kb + mb, z), "iterations gpu", its.tolist(), "oracle", ri.tolist(), "fp64", i64.tolist(),
        "bit errors after decoding", int(np.sum(bits != cw)), "before", int(np.sum(L.hard(llr) != cw)))
    assert np.array_equal(its, ri)
    assert np.array_equal(bits, rb)
    assert np.array_equal(post.view(np.uint32), rp.view(np.uint32))
    # against the FP64 decoder: the same decisions wherever its LLRs are not near zero
    rms = float(np.sqrt(np.mean(r64 ** 2)))
    far = np.abs(r64) > 1e-3 * rms
    say("  fp32 vs fp64: max |d| / RMS", float(np.max(np.abs(post - r64)) / rms), "hard-bit differences away "
        "from zero", int(np.sum((bits != b64) & far)))


def test_ldpc_codewords_and_zero_iterations(rx):
    """A channel word that is already a codeword comes back unchanged with 0
    iterations; max_iter = 0 returns the channel LLRs and their hard bits."""
    z = 48
    base = G.random_base(5, 7, z, 4, seed=51)
    cw = G.make_codewords(base, z, 3, seed=52)
    rng = np.random.default_rng(53)
    clean = ((1.0 - 2.0 * cw) * rng.uniform(0.25, 8.0, cw.shape)).astype(np.float32)
    code = rx.LdpcCode(base, z)
    post, bits, its = (t.cpu().numpy() for t in rx.ldpc_decode(code, torch.from_numpy(clean).cuda(), 10))
    assert np.all(its == 0) and np.array_equal(post, clean) and np.array_equal(bits, cw)
    noisy = G.bpsk_awgn_llrs(cw, 1.0, seed=54)
    post, bits, its = (t.cpu().numpy() for t in rx.ldpc_decode(code, torch.from_numpy(noisy).cuda(), 0))
    assert np.all(its == 0) and np.array_equal(post, noisy) and np.array_equal(bits, L.hard(noisy))


def test_ldpc_lifting_384_sampled(rx):
    """The largest lifting size (z = 384) on a 46 x 68 base matrix (the shape
    of the largest 3GPP base graph, random shifts, N = 26112, posteriors in
    150 KB of LDS): 24 codewords, every one bit for bit against the FP32
    oracle; every codeword whose syndrome reached zero is the transmitted one."""
    z = 384
    base = G.random_base(46, 22, z, 7, seed=61)
    cw = G.make_codewords(base, z, 24, seed=62)
    llr = G.bpsk_awgn_llrs(cw, 2.5, seed=63)
    code = rx.LdpcCode(base, z)
    post, bits, its = (t.cpu().numpy() for t in rx.ldpc_decode(code, torch.from_numpy(llr).cuda(), 6, 0.75))
    say("z 384: iterations", its.tolist(), "codewords in error", int(np.sum(np.any(bits != cw, axis=1))))
    rp, rb, ri = L.decode_batch(base, z, llr, 6, 0.75, dtype=np.float32)
    assert np.array_equal(its, ri) and np.array_equal(bits, rb)
    assert np.array_equal(post.view(np.uint32), rp.view(np.uint32))
    done = np.array([not np.any(L.syndrome_qc(base, z, b)) for b in bits])
    assert np.sum(done) >= 20
    assert np.array_equal(bits[done], cw[done])


def test_ldpc_zero_codewords_is_a_no_op(rx):
    base = G.random_base(3, 3, 8, 2, seed=71)
    code = rx.LdpcCode(base, 8)
    post, bits, its = rx.ldpc_decode(code, torch.empty((0, 48), dtype=torch.float32, device="cuda"))
    assert post.shape == (0, 48) and its.shape == (0,)
