"""Batched uneven frames (one persistent launch, hipGraph replay) against the
single-frame path, frame by frame, and against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import synth
from parity_util import evm_rel, hard_bits_outside_guard, llr_rel, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OUTS = ("yf", "h", "xt", "nu", "flags", "llr")


def say(*a):
    print("[gpu-batch]", *a, flush=True)


def mixed_shapes():
    """Every FFT size, every K padding (4, 8, 16), every modulation, both
    detectors, a cyclic prefix and short frames, plus shapes of the uneven
    256-frame workload."""
    S = synth.Shape
    hand = [(S(8, 1, 512, 300, 14, 0, 2), O.ZF), (S(16, 5, 1024, 777, 14, 16, 4), O.MMSE),
            (S(32, 12, 2048, 1500, 14, 0, 6), O.MMSE), (S(64, 16, 4096, 3276, 14, 0, 4), O.ZF),
            (S(8, 8, 512, 420, 14, 0, 6), O.ZF), (S(64, 3, 4096, 2900, 6, 32, 2), O.MMSE),
            (S(16, 16, 2048, 1700, 17, 0, 2), O.ZF)]
    drawn = [(s, O.MMSE) for s in synth.draw_batch_shapes(7)]
    return hand + drawn


@pytest.fixture(scope="module")
def batch(rx):
    shapes = mixed_shapes()
    inputs = synth.draw_inputs(4, range(len(shapes)), [s for s, _ in shapes], workers=8)
    frames = [rx.Frame.of(s, det, 1.0) for s, det in shapes]
    return frames, inputs


def pack(rx, plan, inputs):
    bufs = plan.alloc()
    for k in ("yf", "h", "xt", "nu", "flags", "llr"):
        bufs[k].fill_(0xEE)
    for f, (x, p) in enumerate(inputs):
        plan.view(bufs, "x", f).copy_(torch.from_numpy(x))
        plan.view(bufs, "pilots", f).copy_(torch.from_numpy(p))
    return bufs


def single(rx, fr, x, p):
    out = rx.forward(fr, torch.from_numpy(x)[None].cuda(), torch.from_numpy(p)[None].cuda())
    return {k: v[0] for k, v in out.items()}


def assert_frames_equal(plan, bufs, refs, frames_idx=None):
    for f in (frames_idx if frames_idx is not None else range(len(plan.frames))):
        for k in OUTS:
            got = plan.view(bufs, k, f)
            ref = refs[f][k]
            same = torch.equal(got, ref) if k not in ("xt", "yf", "h") else \
                torch.equal(torch.view_as_real(got), torch.view_as_real(ref))
            if not same:
                d = (got.to(torch.complex128) - ref.to(torch.complex128)).abs().max().item() \
                    if got.is_complex() else (got.double() - ref.double()).abs().max().item()
                raise AssertionError("frame %d (%s) %s differs, max |diff| %g" % (f, plan.frames[f], k, d))


@pytest.fixture(scope="module")
def refs(rx, batch):
    frames, inputs = batch
    return [single(rx, fr, x, p) for fr, (x, p) in zip(frames, inputs)]


def test_batch_equals_single_frame_path_bitwise(rx, batch, refs):
    frames, inputs = batch
    plan = rx.Plan(frames)
    say("frames", len(frames), "items per stage", plan.counts, "grid", plan.grid)
    bufs = pack(rx, plan, inputs)
    plan.forward(bufs)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert_frames_equal(plan, bufs, refs)


@pytest.mark.parametrize("tiles", [
    dict(fft_iters=1, csi_tiles=1, det_tiles=1, dem_groups=1),
    dict(fft_iters=7, csi_tiles=5, det_tiles=3, dem_groups=33),
    dict(fft_iters=64, csi_tiles=512, det_tiles=256, dem_groups=4096),
])
def test_batch_tile_sizes_do_not_change_results(rx, batch, refs, tiles):
    frames, inputs = batch
    plan = rx.Plan(frames, tiles=rx.Tiles(**tiles))
    say(tiles, "items", plan.counts)
    bufs = pack(rx, plan, inputs)
    plan.forward(bufs)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert_frames_equal(plan, bufs, refs)


def assert_fused_frames_equal(plan, bufs, refs, frames_idx=None):
    """A plan that forms the channel estimate (and / or demaps) inside the
    detector items: every output it writes (all but H, and x_tilde when the
    demod is fused) equals the single-frame (staged) calls bit for bit."""
    keys = [k for k in ("yf", "xt", "nu", "flags", "llr") if not (k == "xt" and plan.fuse_demod)]
    for f in (frames_idx if frames_idx is not None else range(len(plan.frames))):
        for k in keys:
            got, ref = plan.view(bufs, k, f), refs[f][k]
            same = torch.equal(torch.view_as_real(got), torch.view_as_real(ref)) if got.is_complex() else \
                torch.equal(got, ref)
            assert same, "frame %d (%s) %s differs" % (f, plan.frames[f], k)


@pytest.mark.parametrize("tiles", [None, dict(fft_iters=1, det_tiles=1, dem_groups=1),
                                   dict(fft_iters=13, det_tiles=5, dem_groups=29)])
def test_batch_fused_csi_equals_staged_and_single_frame_fused_calls(rx, batch, refs, tiles):
    """fuse_csi: no CSI items, H never written (its buffer is a one-byte
    placeholder), detector items wait for the FFT items of their frame; the
    outputs equal the staged calls bit for bit, and, frame by frame, the fused
    single-frame calls rxphy_csi_detect + rxphy_demod where those take the
    same per-subcarrier path (fewer than 16 users; with 16 users the
    single-frame fused call factors each pilot group once, whose x_tilde
    differs in the last bits: there nu and flags are equal and, where the
    channel is well-conditioned (M >= 2K), the LLRs within the stated
    tolerance)."""
    frames, inputs = batch
    plan = rx.Plan(frames, tiles=rx.Tiles(**tiles) if tiles else None, fuse_csi=True)
    say("fused", tiles, "items", plan.counts, "grid", plan.grid)
    assert plan.counts[1] == 0
    bufs = pack(rx, plan, inputs)
    assert bufs["h"].numel() == 1
    plan.forward(bufs)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert_fused_frames_equal(plan, bufs, refs)
    if tiles is None:
        for f, fr in enumerate(frames):
            yf = plan.view(bufs, "yf", f)[None]
            p = plan.view(bufs, "pilots", f)[None]
            xt, nu, fl = rx.csi_detect(fr, yf, p)
            llr = rx.demod(fr, xt, nu)
            if fr.K < 16:
                assert torch.equal(torch.view_as_real(xt[0]), torch.view_as_real(plan.view(bufs, "xt", f)))
                assert torch.equal(llr[0], plan.view(bufs, "llr", f))
            elif fr.M >= 2 * fr.K:                # well-conditioned; square ZF channels reach kappa ~ 1e5
                lr = llr_rel(plan.view(bufs, "llr", f).cpu().numpy(), llr[0].cpu().numpy())
                assert lr < 1e-3, (f, lr)
            assert torch.equal(nu[0], plan.view(bufs, "nu", f)) and torch.equal(fl[0], plan.view(bufs, "flags", f))


@pytest.mark.parametrize("fuse_csi", [True, False])
@pytest.mark.parametrize("tiles", [None, dict(fft_iters=1, det_tiles=1), dict(fft_iters=13, det_tiles=5)])
def test_batch_fused_demod_equals_staged(rx, batch, refs, fuse_csi, tiles):
    """fuse_demod: no demod items; each detector item demaps its tiles from
    x_tilde and nu held in LDS, which is never written to memory (its buffer
    is a one-byte placeholder); LLRs, nu and flags equal the staged calls bit
    for bit, with and without the CSI stage fused in, for several item sizes
    (tiles of several detector tiles per item reuse the LDS between tiles)."""
    frames, inputs = batch
    plan = rx.Plan(frames, tiles=rx.Tiles(**tiles) if tiles else None, fuse_csi=fuse_csi, fuse_demod=True)
    say("fused demod", "csi fused" if fuse_csi else "csi items", tiles, "items", plan.counts)
    assert plan.counts[3] == 0 and (plan.counts[1] == 0) == fuse_csi
    bufs = pack(rx, plan, inputs)
    assert bufs["xt"].numel() == 1
    plan.forward(bufs)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert_fused_frames_equal(plan, bufs, refs)


def test_batch_wider_k_padding_within_tolerance(rx, batch, refs):
    frames, inputs = batch
    plan = rx.Plan(frames, tiles=rx.Tiles(det_kp=16))
    bufs = pack(rx, plan, inputs)
    plan.forward(bufs)
    torch.cuda.synchronize()
    for f, fr in enumerate(frames):
        xt = plan.view(bufs, "xt", f).cpu().numpy()
        ref = refs[f]["xt"].cpu().numpy()
        e = evm_rel(xt, ref, np.ones(fr.n_sc, bool))
        lr = llr_rel(plan.view(bufs, "llr", f).cpu().numpy(), refs[f]["llr"].cpu().numpy())
        assert e < 1e-5 and lr < 1e-3, (f, fr, e, lr)
        assert torch.equal(plan.view(bufs, "flags", f), refs[f]["flags"])


def test_batch_one_workgroup_and_odd_grids(rx, batch, refs):
    frames, inputs = batch
    for grid in (1, 3, 1000):
        plan = rx.Plan(frames[:5], grid=grid)
        bufs = pack(rx, plan, inputs[:5])
        plan.forward(bufs)
        torch.cuda.synchronize()
        say("grid", grid, "status", plan.device_status())
        assert plan.device_status() == 0
        assert_frames_equal(plan, bufs, refs, range(5))


def test_batch_stage_masks_compose(rx, batch, refs):
    frames, inputs = batch
    p1 = rx.Plan(frames, stages=rx.STAGE_FFT | rx.STAGE_CSI)
    p2 = rx.Plan(frames, stages=rx.STAGE_DETECT | rx.STAGE_DEMOD)
    assert p1.counts[2] == 0 and p2.counts[0] == 0
    bufs = pack(rx, p1, inputs)
    p1.forward(bufs)
    p2.forward(bufs)
    torch.cuda.synchronize()
    assert_frames_equal(p2, bufs, refs)


@pytest.mark.parametrize("fuse", [False, True, "full"])
def test_batch_graph_replays_match_eager(rx, batch, refs, fuse):
    frames, inputs = batch
    plan = rx.Plan(frames, fuse_csi=bool(fuse), fuse_demod=fuse == "full")
    bufs = pack(rx, plan, inputs)
    plan.graph(bufs)
    for rep in range(3):
        for k in ("yf", "h", "xt", "nu", "flags", "llr"):
            bufs[k].zero_()
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        say("replay", rep, "fused" if fuse else "staged", "status", plan.device_status())
        assert plan.device_status() == 0
        if fuse:
            assert_fused_frames_equal(plan, bufs, refs)
        else:
            assert_frames_equal(plan, bufs, refs)
        # the program's own eager work between replays
        single(rx, frames[0], *inputs[0])
        torch.cuda.synchronize()


def test_batch_matches_oracle(rx, batch):
    frames, inputs = batch
    plan = rx.Plan(frames)
    bufs = pack(rx, plan, inputs)
    plan.forward(bufs)
    torch.cuda.synchronize()
    for f in (0, 1, 5, 8):
        fr = frames[f]
        sh = synth.Shape(fr.M, fr.K, fr.n_fft, fr.n_sc, fr.n_sym, fr.cp_len, fr.qam_bits)
        x, p = inputs[f]
        ref = O.forward(x, p, sh, fr.n0, fr.detector, want_kappa=True)
        good = (ref["kappa"] <= 1e3) & (ref["flags"] == 0)
        e = evm_rel(plan.view(bufs, "xt", f).cpu().numpy(), ref["xt"], good)
        llr = plan.view(bufs, "llr", f).cpu().numpy()
        lr = llr_rel(llr, ref["llr"])
        mism, band = hard_bits_outside_guard(llr, ref["llr"])
        say("frame", f, fr, "evm_rel", e, "llr_rel", lr, "hard-bit mismatches", mism, "in band", band)
        assert e < 1e-4 and lr < 1e-3 and mism == 0
        assert rel_rms(plan.view(bufs, "yf", f).cpu().numpy(), ref["yf"]) < 1e-5


@pytest.mark.parametrize("fuse", ["full", True, False])
def test_batch_uneven_256_frames_full_size(rx, fuse):
    """The 256-frame uneven workload in the launch configurations the
    benchmark times (the channel estimate formed and the tiles demapped inside
    the detector items; the estimate alone; the staged dataflow); sampled
    frames are compared with the single-frame path."""
    shapes = synth.draw_batch_shapes(256)
    frames = [rx.Frame.of(s, O.MMSE, 1.0) for s in shapes]
    plan = rx.Plan(frames, fuse_csi=bool(fuse), fuse_demod=fuse == "full")
    say("256 frames, items", plan.counts, "grid", plan.grid,
        "x GB", round(plan.totals["x"] / 1e9, 3))
    bufs = plan.alloc()
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    # received samples: Rayleigh-faded QAM-like signal energy plus noise, drawn
    # on the device (the comparison is path against path)
    for k in ("x", "pilots"):
        n = plan.totals[k] // 8
        v = torch.randn((n, 2), generator=g, device="cuda", dtype=torch.float32)
        bufs[k][: n * 8].view(torch.float32).copy_(v.view(-1))
    plan.graph(bufs)
    plan.replay()
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    for f in (0, 1, 77, 128, 200, 255):
        fr = frames[f]
        x = plan.view(bufs, "x", f)[None].contiguous()
        p = plan.view(bufs, "pilots", f)[None].contiguous()
        ref = rx.forward(fr, x, p)
        for k in OUTS:
            if (fuse and k == "h") or (fuse == "full" and k == "xt"):
                continue
            a, b = plan.view(bufs, k, f), ref[k][0]
            if a.is_complex():
                a, b = torch.view_as_real(a), torch.view_as_real(b)
            assert torch.equal(a, b), (f, fr, k)


def test_autotuned_tiles_keep_results_bitwise(rx, batch, refs, tmp_path):
    from paper_2603_20481_amd.autotune import Tuner
    frames, inputs = batch
    t = Tuner(str(tmp_path / "tiles.json"))
    info = t.tune(frames, copies=4, reps=2)
    say("autotune", info, "entries", len(t.entries))
    assert info["classes_tuned"] == len(t.entries) > 0
    t.save()
    t2 = Tuner(str(tmp_path / "tiles.json"))
    assert t2.tune(frames)["classes_tuned"] == 0          # everything cached
    plan = rx.Plan(frames, tiles=t2.tiles_for(frames), fuse_csi=True, fuse_demod=True)
    bufs = pack(rx, plan, inputs)
    plan.forward(bufs)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert_fused_frames_equal(plan, bufs, refs)
    # the plan-wide knobs: every candidate dataflow and grid gives the same outputs
    bufs = pack(rx, rx.Plan(frames), inputs)              # with an H buffer: staged candidates run too
    pick = t2.tune_plan(frames, bufs, reps=2)
    say("plan knobs", pick)
    assert pick["item_sizes"] in ("tuned", "default") and len(pick["candidates_us"]) == 24
    plan = rx.Plan(frames, tiles=pick["tiles"], grid=pick["grid"], fuse_csi=pick["fuse_csi"],
                   fuse_demod=pick["fuse_demod"])
    bufs = pack(rx, plan, inputs)
    plan.forward(bufs)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert_fused_frames_equal(plan, bufs, refs)
