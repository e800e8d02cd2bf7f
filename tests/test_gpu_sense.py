"""GPU parity of the sensing pipeline (rxphy_sense) against the oracle, stage
by stage on the GPU's own upstream results: the TF plot against the FP64
transform; the PSD and its smoothing within FP32 summation error; the noise
floor as the exact lowest local minimum of the GPU's smoothed PSD; theta in
FP32; the Otsu bins, the mask, the morphology and the boxes bit for bit
(integer work, with every floating-point decision taken in FP32 on both
sides)."""
import numpy as np
import pytest

from oracle import sensing_oracle as S
from synth import sensing as SS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-sense]", *a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b ** 2), 1e-300)))


def check_plot(cfg, ocfg, x, g, i, max_boxes):
    tf = g["tf"][i]
    assert rel(tf, S.tf_plot(x, cfg.n_fft)) < 2e-6
    psd = g["psd"][i]
    assert rel(psd, S.psd(tf)) < 2e-6
    ps = g["psd_smooth"][i]
    assert rel(ps, S.sg_smooth(psd, cfg.sg_window, cfg.sg_order)) < 2e-6
    n0, theta = g["floor"][i]
    assert n0 == S.noise_floor(ps.astype(np.float64))          # a selection: exact
    assert theta == np.float32(cfg.psd_factor) * n0            # FP32 product
    retained = psd >= theta                                    # FP32 comparison
    mask, ks = S.binarize(tf, retained, cfg.bins)
    assert np.array_equal(g["otsu_bin"][i], ks)
    assert np.array_equal(g["mask"][i], mask)
    mo = S.morph(g["mask"][i])
    assert np.array_equal(g["mask_mo"][i], mo)
    bx = S.boxes(g["mask_mo"][i])
    assert g["n_boxes"][i] == len(bx)
    k = min(len(bx), max_boxes)
    assert np.array_equal(g["boxes"][i][:k], bx[:k])
    return retained, bx


CASES = [  # (F, T, scenario, plots, max_boxes)
    (512, 400, "sparse_wifi", 2, 64),
    (1024, 2000, "mixed", 2, 256),
    (1024, 333, "dense_ble", 3, 256),                         # T not a multiple of 64
    (2048, 150, "dense_wifi", 1, 256),
    (1024, 2000, "dense_ble", 1, 5),                          # more components than box slots
]


@pytest.mark.parametrize("F,T,scen,P,max_boxes", CASES)
def test_sense_stages_vs_oracle(rx, F, T, scen, P, max_boxes):
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    ocfg = S.SenseConfig(F=F, T=T)
    scenes = [SS.make_scene(100 + s, scen, T=T, F=F) for s in range(P)]
    x = torch.from_numpy(np.stack([s.x for s in scenes])).cuda()
    out = rx.sense(cfg, x, max_boxes=max_boxes, intermediates=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    for i, sc in enumerate(scenes):
        retained, bx = check_plot(cfg, ocfg, sc.x, g, i, max_boxes)
        m = S.metrics(sc.boxes, bx, 0.4)
        say(F, T, scen, "plot", i, "retained", int(retained.sum()), "boxes", len(bx), "gt", len(sc.boxes),
            "P_d %.2f P_fa %.2f mean IoU %.2f" % (m["p_d"], m["p_fa"], m["mean_iou"]))


def test_sense_configs_and_degenerate_plots(rx):
    """Other Savitzky-Golay orders, bin counts and factors; an all-zero plot
    (no threshold anywhere, no boxes); a plot whose every column is retained."""
    T, F = 256, 512
    sc = SS.make_scene(7, "dense_wifi", T=T, F=F)
    zero = np.zeros((T, F), np.complex64)
    rng = np.random.default_rng(3)
    loud = (rng.standard_normal((T, F)) + 1j * rng.standard_normal((T, F))).astype(np.complex64)
    loud[T // 3: T // 2] *= 30                                # a wideband burst: every column retained
    x = torch.from_numpy(np.stack([sc.x, zero, loud])).cuda()
    for cfg in (rx.SenseConfig(n_fft=F, n_rows=T, sg_order=3, psd_factor=1.05, bins=64),
                rx.SenseConfig(n_fft=F, n_rows=T, sg_window=3, sg_order=0, psd_factor=1.2, bins=2),
                rx.SenseConfig(n_fft=F, n_rows=T, sg_window=63, sg_order=6, psd_factor=1.1, bins=256)):
        out = rx.sense(cfg, x, max_boxes=128, intermediates=True)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
        ocfg = S.SenseConfig(F=F, T=T, sg_window=cfg.sg_window, sg_order=cfg.sg_order,
                             psd_factor=cfg.psd_factor, bins=cfg.bins)
        for i, xi in enumerate((sc.x, zero, loud)):
            retained, bx = check_plot(cfg, ocfg, xi, g, i, 128)
            say("cfg", cfg.sg_window, cfg.sg_order, cfg.psd_factor, cfg.bins, "plot", i,
                "retained", int(retained.sum()), "boxes", len(bx))
        assert g["n_boxes"][1] == 0 and not g["mask"][1].any()
        assert (g["otsu_bin"][1] == -1).all()


def test_sense_is_deterministic_and_reuses_workspace(rx):
    T, F = 2000, 1024
    scenes = [SS.make_scene(50 + s, "mixed", T=T, F=F) for s in range(2)]
    x = torch.from_numpy(np.stack([s.x for s in scenes])).cuda()
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    ws = torch.empty((rx.sense_workspace_bytes(cfg, 2),), dtype=torch.uint8, device="cuda")
    a = rx.sense(cfg, x, max_boxes=256, ws=ws)
    b = rx.sense(cfg, x, max_boxes=256, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(a["n_boxes"], b["n_boxes"]) and torch.equal(a["boxes"], b["boxes"])


@pytest.mark.parametrize("F,T", [(4096, 70), (512, 3), (1024, 65)])
def test_sense_edge_shapes_and_no_box_array(rx, F, T):
    """The widest plot, the fewest rows (3) and a single row past one tile,
    on noise with a strong block; then the same call with max_boxes = 0 (no
    box array), which still counts the components."""
    rng = np.random.default_rng([41, F, T])
    x = ((rng.standard_normal((2, T, F)) + 1j * rng.standard_normal((2, T, F))) / np.sqrt(2)).astype(np.complex64)
    blk = np.zeros((T, F), np.complex128)
    cols = (np.arange(F // 8, F // 4) - F // 2) % F
    blk[:, cols] = (rng.standard_normal((T, len(cols))) + 1j * rng.standard_normal((T, len(cols)))) * np.sqrt(F * 50)
    x[1] += np.fft.ifft(blk, axis=1).astype(np.complex64)
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    ocfg = S.SenseConfig(F=F, T=T)
    xd = torch.from_numpy(x).cuda()
    out = rx.sense(cfg, xd, max_boxes=64, intermediates=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    for i in range(2):
        retained, bx = check_plot(cfg, ocfg, x[i], g, i, 64)
        say("edge", F, T, "plot", i, "retained", int(retained.sum()), "boxes", len(bx))
    none = rx.sense(cfg, xd, max_boxes=0)
    torch.cuda.synchronize()
    assert np.array_equal(none["n_boxes"].cpu().numpy(), g["n_boxes"])


def test_sense_bench_launch_sampled_plots(rx):
    """64 plots of (2000, 1024) in one call, as the benchmark launches them
    (16 distinct scenes repeated); sampled plots checked stage by stage, and
    every repeat of a scene gives the same boxes."""
    T, F, P = 2000, 1024, 64
    scenes = [SS.make_scene(900 + i, "mixed", T=T, F=F) for i in range(16)]
    x = torch.from_numpy(np.stack([scenes[i % 16].x for i in range(P)])).cuda()
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    ocfg = S.SenseConfig(F=F, T=T)
    out = rx.sense(cfg, x, max_boxes=1024, intermediates=True)
    torch.cuda.synchronize()
    nb = out["n_boxes"].cpu().numpy()
    bx = out["boxes"].cpu().numpy()
    for i in range(16, P):
        assert nb[i] == nb[i % 16] and np.array_equal(bx[i], bx[i % 16])
    for i in (0, 37, 63):
        g = {k: v[i:i + 1].cpu().numpy() for k, v in out.items()}
        retained, b = check_plot(cfg, ocfg, scenes[i % 16].x, g, 0, 1024)
        say("64-plot launch, plot", i, "retained", int(retained.sum()), "boxes", len(b))


def lattice_capture(T, F, period=6, size=3, offset=2, big=100.0, small=1.0):
    """Samples whose TF plot is a lattice of size x size blocks (gaps of
    period - size, which the 3x3 closing does not bridge): every 64x64 tile
    then holds up to 121 components."""
    cols = (np.arange(F) - F // 2) % F
    on_t = ((np.arange(T) - offset) % period) < size
    on_f = ((np.arange(F) - offset) % period) < size
    X = np.where(on_t[:, None] & on_f[None, :], big, small).astype(np.complex128)
    Xb = np.zeros((T, F), np.complex128)
    Xb[:, cols] = X
    return np.fft.ifft(Xb, axis=1).astype(np.complex64), on_t[:, None] & on_f[None, :]


def test_sense_dense_lattice_overflows_the_tile_lists(rx):
    """More components per tile than a tile's list holds: the box kernel reads
    those tiles pixel by pixel and still returns the oracle's boxes."""
    T, F = 200, 512
    x, lat = lattice_capture(T, F)
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    ocfg = S.SenseConfig(F=F, T=T)
    out = rx.sense(cfg, torch.from_numpy(x[None]).cuda(), max_boxes=4096, intermediates=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    retained, bx = check_plot(cfg, ocfg, x, g, 0, 4096)
    say("lattice", T, F, "boxes", len(bx), "mask equals lattice", bool(np.array_equal(g["mask_mo"][0], lat)))
    assert np.array_equal(g["mask_mo"][0], lat.astype(np.uint8))
    assert len(bx) > 64 * (T // 64) * (F // 64) // 4


def test_sense_components_across_listed_and_overflowed_tiles(rx):
    """Lattice tiles (lists overflowed, resolved pixel by pixel) next to
    tiles with component lists, with components that cross between them in
    both directions (first pixel in a listed tile with pixels in overflowed
    tiles, and the reverse), and a partial last tile row: boxes equal the
    oracle's."""
    ndimage = pytest.importorskip("scipy.ndimage")
    T, F = 250, 512
    t, f = np.arange(T)[:, None], np.arange(F)[None, :]
    on = (((t - 2) % 6) < 3) & (((f - 2) % 6) < 3) & (t >= 64) & (f < 256)
    on[150:171, 0:421] = True                    # band from the lattice into listed tiles
    on[40:71, 200:301] = True                    # first pixel in a listed tile, reaches the lattice
    on[20:51, 300:401] = True
    on[180:241, 440:481] = True
    cols = (np.arange(F) - F // 2) % F
    Xb = np.zeros((T, F), np.complex128)
    Xb[:, cols] = np.where(on, 100.0, 1.0)
    x = np.fft.ifft(Xb, axis=1).astype(np.complex64)
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    ocfg = S.SenseConfig(F=F, T=T)
    out = rx.sense(cfg, torch.from_numpy(x[None]).cuda(), max_boxes=2048, intermediates=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    retained, bx = check_plot(cfg, ocfg, x, g, 0, 2048)
    mo = g["mask_mo"][0].astype(bool)
    ov = np.zeros((T, F), bool)
    for ty in range(0, T, 64):
        for tx in range(0, F, 64):
            ov[ty:ty + 64, tx:tx + 64] = ndimage.label(mo[ty:ty + 64, tx:tx + 64])[1] > 64
    lab, nc = ndimage.label(mo)
    kinds = set()
    for c in range(1, nc + 1):
        pix = np.argwhere(lab == c)
        o = ov[pix[:, 0], pix[:, 1]]
        if o.any() and (~o).any():
            kinds.add(bool(ov[pix[0][0], pix[0][1]]))
    say("mixed lattice", T, F, "boxes", len(bx), "overflowed tiles", int(ov[::64, ::64].sum()), "crossings", kinds)
    assert 0 < ov[::64, ::64].sum() < ov[::64, ::64].size
    assert kinds == {True, False}


def test_sense_largest_plot_many_components(rx):
    """The largest plot (4096 x 4096): lattice squares on a checkerboard of
    512 x 512 regions (tiles with overflowed and with listed components) and
    a band across them, about 227,000 components, so the ordinal scan runs
    over every one of its 262,144 counts; every box equals the oracle's."""
    T = F = 4096
    t, f = np.arange(T)[:, None], np.arange(F)[None, :]
    on = (((t - 2) % 6) < 3) & (((f - 2) % 6) < 3) & ((t // 512 + f // 512) % 2 == 0)
    on[1000:1100, 100:4000] = True
    cols = (np.arange(F) - F // 2) % F
    Xb = np.zeros((T, F), np.complex128)
    Xb[:, cols] = np.where(on, 100.0, 1.0)
    x = np.fft.ifft(Xb, axis=1).astype(np.complex64)
    del Xb
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    ocfg = S.SenseConfig(F=F, T=T)
    mb = 1 << 18
    out = rx.sense(cfg, torch.from_numpy(x[None]).cuda(), max_boxes=mb, intermediates=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    retained, bx = check_plot(cfg, ocfg, x, g, 0, mb)
    say("largest plot", T, F, "boxes", len(bx))
    assert 100_000 < len(bx) < mb
