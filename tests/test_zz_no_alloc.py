"""The allocation-free fused call (rxphy_csi_detect_demod_noalloc, the
library's per-GPU scratch as its workspace) against rxphy_csi_detect_demod
with a caller-allocated workspace: bit-identical LLRs, noise variances, flags
and equalised symbols, on two calls in a row with the second one smaller
(the scratch keeps the first call's contents), for the 16-user FP32 path
(per-tile factor records in the scratch), the general FP32 path (x_tilde
staged in the scratch) and the BF16 path (refinement list in the scratch),
and at the largest frame count the scratch holds."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)


def _frames(rx, shape, n, det, seed):
    frs = [synth.make_frame(seed, f, shape=shape) for f in range(n)]
    fr = rx.Frame.of(shape, det, 1.0)
    x = torch.from_numpy(np.stack([f.x for f in frs])).cuda()
    p = torch.from_numpy(np.stack([f.pilots for f in frs])).cuda()
    return fr, rx.fft(fr, x), p


def _same(a, b, what):
    for name, u, v in zip(("llr", "nu", "flags", "xt"), a, b):
        if u is None and v is None:
            continue
        assert torch.equal(u, v), "%s: %s differs" % (what, name)


CASES = [
    # shape of the first call, frames of the first and second call, detector, precision
    ("64x16 fp32", synth.Shape(64, 16, 2048, 1200, 14, 0, 4), (3, 1), 0, "fp32"),
    ("32x8 fp32", synth.Shape(32, 8, 1024, 601, 14, 0, 6), (2, 1), 1, "fp32"),
    ("16x5 bf16", synth.Shape(16, 5, 512, 300, 14, 0, 2), (2, 1), 0, "bf16"),
]


@pytest.mark.parametrize("name,shape,counts,det,prec", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_workspace_call_twice(rx, name, shape, counts, det, prec):
    for k, n in enumerate(counts):
        say(name, "call", k + 1, "frames", n)
        fr, yf, p = _frames(rx, shape, n, det, 40 + k)
        want_xt = k == 0
        ref = rx.csi_detect_demod(fr, yf, p, prec, 1e3, want_xt=want_xt)
        xt = torch.empty_like(ref[3]) if want_xt else None
        got = rx.csi_detect_demod_noalloc(fr, yf, p, prec, 1e3, xt=xt)
        torch.cuda.synchronize()
        _same(got, ref, "%s call %d" % (name, k + 1))
        if prec == "bf16":
            say("  refined subcarriers", int((ref[2] == 1).sum()))


def test_noalloc_at_the_scratch_limit_then_small(rx):
    """194 frames of 64 x 16 with 1200 subcarriers (the most the 32 MiB scratch
    holds on the 16-user path), then 2 frames: random unit-power data with
    unit-modulus pilots, compared with the workspace call."""
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    for n in (194, 2):
        say("scratch limit case, frames", n)
        fr = rx.Frame(64, 16, 2048, 1200, 14, 0, 4, 0, 1.0)
        yf = torch.randn((n, 64, 14, 1200), dtype=torch.complex64, device="cuda", generator=g)
        ph = torch.rand((n, 1200), device="cuda", generator=g) * 6.283185307179586
        p = torch.polar(torch.ones_like(ph), ph).to(torch.complex64)
        assert rx.workspace_bytes(fr, n, rx.WS_CSI_DETECT_DEMOD) <= 32 << 20
        ref = rx.csi_detect_demod(fr, yf, p)
        got = rx.csi_detect_demod_noalloc(fr, yf, p)
        torch.cuda.synchronize()
        _same(got, ref, "%d frames" % n)
        del yf, ref, got
