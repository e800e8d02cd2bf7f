"""Pins of the sensing oracle (CPU): each step against something other than
itself -- a term-by-term DFT, scipy's Savitzky-Golay routines, brute-force
Otsu over exact fractions, scipy.ndimage's morphology and labelling, and
hand-worked examples of the detection metrics (Section III-A)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.signal as sig

from oracle import sensing_oracle as S
from synth import sensing as SS


def test_tf_plot_term_by_term_dft_and_centred_columns():
    rng = np.random.default_rng(1)
    T, F = 3, 8
    x = rng.standard_normal((T, F)) + 1j * rng.standard_normal((T, F))
    tf = S.tf_plot(x, F)
    for t in range(T):
        for c in range(F):
            k = (c - F // 2) % F
            X = sum(x[t, n] * np.exp(-2j * np.pi * k * n / F) for n in range(F))
            assert tf[t, c] == pytest.approx(abs(X), rel=1e-12)
    # a tone at bin k lands in column (k + F/2) mod F with magnitude F
    F = 64
    for k in (0, 1, 5, 31, 32, 63):
        tone = np.exp(2j * np.pi * k * np.arange(F) / F)[None]
        row = S.tf_plot(tone, F)[0]
        assert row.argmax() == (k + F // 2) % F and row.max() == pytest.approx(F)
        assert np.sum(row) == pytest.approx(F, abs=1e-9 * F)


def test_psd_is_the_time_sum():
    tf = np.arange(12, dtype=float).reshape(4, 3)
    assert np.array_equal(S.psd(tf), [18, 22, 26])


@pytest.mark.parametrize("w,o", [(21, 3), (5, 2), (31, 4), (7, 0), (9, 6)])
def test_savitzky_golay_matches_scipy(w, o):
    assert np.allclose(S.sg_coeffs(w, o), sig.savgol_coeffs(w, o), rtol=1e-10, atol=1e-12)
    rng = np.random.default_rng(w * 10 + o)
    p = rng.standard_normal(300).cumsum()
    assert np.allclose(S.sg_smooth(p, w, o), sig.savgol_filter(p, w, o, mode="mirror"), rtol=1e-10, atol=1e-10)
    # a polynomial of degree <= order passes unchanged away from the edges
    j = np.arange(100, dtype=float)
    poly = 0.3 - 0.2 * j + (0.01 * j ** 2 if o >= 2 else 0) + (1e-4 * j ** 3 if o >= 3 else 0)
    if o >= 1:
        h = w // 2
        assert np.allclose(S.sg_smooth(poly, w, o)[h:-h], poly[h:-h], rtol=1e-9, atol=1e-9)


def test_mirror_index():
    n = 5
    assert [S.mirror_index(j, n) for j in range(-4, 9)] == [4, 3, 2, 1, 0, 1, 2, 3, 4, 3, 2, 1, 0]


def test_noise_floor_lowest_local_minimum():
    assert S.noise_floor([3, 1, 2, 0.5, 4]) == 0.5
    assert S.noise_floor([0, 1, 2, 3, 2.5, 5]) == 2.5       # the edge value is no local minimum
    assert S.noise_floor([2, 1, 1, 2]) == 1
    assert S.noise_floor([1, 2, 3]) == 1                    # none: the smallest value
    rng = np.random.default_rng(4)
    for _ in range(50):
        s = rng.standard_normal(40)
        n0 = S.noise_floor(s)
        j = int(np.flatnonzero(s == n0)[0])
        assert 0 < j < 39 and s[j] <= s[j - 1] and s[j] <= s[j + 1]       # a local minimum
        loc = (s[1:-1] <= s[:-2]) & (s[1:-1] <= s[2:])
        assert n0 == s[1:-1][loc].min()                                  # and the lowest one
        if 0 < s.argmin() < 39:
            assert n0 == s.min()                                         # an interior global minimum


def otsu_fraction(h):
    """Otsu from its definition with exact fractions: class weights and means."""
    h = [int(v) for v in h]
    N = sum(h)
    best, best_k = None, -1
    for k in range(len(h) - 1):
        w0 = Fraction(sum(h[:k + 1]), N)
        w1 = 1 - w0
        if w0 == 0 or w1 == 0:
            continue
        mu0 = Fraction(sum(i * h[i] for i in range(k + 1)), sum(h[:k + 1]))
        mu1 = Fraction(sum(i * h[i] for i in range(k + 1, len(h))), sum(h[k + 1:]))
        var = w0 * w1 * (mu0 - mu1) ** 2
        if best is None or var > best:
            best, best_k = var, k
    return best_k


def test_otsu_matches_the_definition_exactly():
    rng = np.random.default_rng(5)
    for trial in range(300):
        bins = int(rng.integers(2, 12))
        n = int(rng.integers(1, 40))
        b = rng.integers(0, bins, n)
        h = np.bincount(b, minlength=bins)
        assert S.otsu_threshold(b, bins) == otsu_fraction(h), (trial, h)
    assert S.otsu_threshold([0] * 5 + [2] * 5, 3) == 0      # tie: the smallest k
    assert S.otsu_threshold([3] * 7, 8) == -1                # one bin occupied: no threshold
    # two separated modes are split between them
    b = np.r_[np.full(100, 10), np.full(30, 200)]
    k = S.otsu_threshold(b, 256)
    assert 10 <= k < 200


def test_column_bins_fp32():
    v = np.float32([1.0, 2.0, 3.0, 5.0, 1.5])
    b, lo, hi = S.column_bins(v, 4)
    assert (lo, hi) == (1.0, 5.0)
    assert list(b) == [0, 1, 2, 3, 0]                        # the maximum lands in the last bin
    rng = np.random.default_rng(6)
    v = rng.gamma(2.0, 3.0, 500).astype(np.float32)
    b, lo, hi = S.column_bins(v, 256)
    scale = np.float32(256) / np.float32(hi - lo)
    for i in range(0, 500, 7):
        d = np.float32(v[i] - lo)
        assert b[i] == min(255, int(np.floor(np.float32(d * scale))))
    b, _, _ = S.column_bins(np.full(9, 2.5, np.float32), 256)
    assert not b.any()


def test_binarize_columns():
    T = 200
    rng = np.random.default_rng(7)
    tf = rng.rayleigh(1.0, (T, 6)).astype(np.float32)
    tf[50:80, 2] += 20.0                                    # a strong burst in column 2
    retained = np.array([True, True, True, False, True, True])
    mask, ks = S.binarize(tf, retained, 256)
    assert ks[3] == -1 and not mask[:, 3].any()
    assert mask[50:80, 2].all() and not mask[:50, 2].any() and not mask[80:, 2].any()


def test_morphology_matches_scipy():
    rng = np.random.default_rng(8)
    for trial in range(20):
        a = (rng.random((40, 37)) < rng.uniform(0.2, 0.8)).astype(np.uint8)
        se = np.ones((3, 3), bool)
        sh = np.ones((1, 3), bool)
        assert np.array_equal(S.dilate(a, 1, 1), ndi.binary_dilation(a, se, border_value=0))
        assert np.array_equal(S.erode(a, 1, 1), ndi.binary_erosion(a, se, border_value=1))
        assert np.array_equal(S.erode(a, 0, 1), ndi.binary_erosion(a, sh, border_value=1))
        ref = ndi.binary_erosion(ndi.binary_dilation(a, se, border_value=0), se, border_value=1)
        ref = ndi.binary_dilation(ndi.binary_erosion(ref, se, border_value=1), se, border_value=0)
        ref = ndi.binary_dilation(ndi.binary_erosion(ref, sh, border_value=1), sh, border_value=0)
        assert np.array_equal(S.morph(a), ref)
        # a 1x3 opening after the 3x3 opening is the identity
        o3 = ndi.binary_dilation(ndi.binary_erosion(a, se, border_value=1), se, border_value=0)
        assert np.array_equal(ndi.binary_dilation(ndi.binary_erosion(o3, sh, border_value=1), sh, border_value=0), o3)


def test_morphology_effects():
    a = np.zeros((20, 20), np.uint8)
    a[5, 5] = 1                                              # isolated pixel: removed
    a[10:15, 2:12] = 1
    a[12, 6] = 0                                             # a hole: filled
    a[2:18, 17] = 1                                          # one bin wide: removed
    m = S.morph(a)
    assert not m[5, 5] and m[12, 6] and not m[:, 17].any()
    assert m[10:15, 2:12].all()
    full = np.ones((6, 6), np.uint8)
    assert S.morph(full).all()                               # the plot edge erodes nothing
    # two blocks with a one-bin line in the three-bin gap between them: the
    # closing bridges the one-bin gaps on both sides, one block results
    b = np.zeros((12, 15), np.uint8)
    b[2:10, 0:5] = 1
    b[2:10, 8:13] = 1
    b[2:10, 6] = 1
    m = S.morph(b)
    assert m[3:9, 0:13].all() and len(S.boxes(m)) == 1


def test_boxes_match_scipy_label():
    rng = np.random.default_rng(9)
    for trial in range(20):
        a = ndi.binary_opening(rng.random((60, 70)) < 0.45).astype(np.uint8)
        lab, n = ndi.label(a)                               # default structure: 4-connectivity
        sl = ndi.find_objects(lab)
        first = [np.flatnonzero(lab.ravel() == k + 1)[0] for k in range(n)]
        ref = [(sl[k][0].start, sl[k][1].start, sl[k][0].stop - 1, sl[k][1].stop - 1)
               for k in np.argsort(first)]
        got = S.boxes(a)
        assert [tuple(b) for b in got] == ref
    assert S.boxes(np.zeros((4, 4), np.uint8)).shape == (0, 4)
    d = np.zeros((3, 3), np.uint8)
    d[0, 0] = d[1, 1] = 1                                    # diagonal: two components
    assert len(S.boxes(d)) == 2


def test_metrics_worked_example():
    gt = [(0, 0, 9, 9)]
    det = [(0, 0, 9, 4), (20, 20, 21, 21)]
    assert S.iou(gt[0], det[0]) == 0.5 and S.iou(gt[0], det[1]) == 0.0
    m = S.metrics(gt, det, 0.4)
    assert (m["n_t"], m["n_f"], m["p_d"], m["p_fa"], m["mean_iou"]) == (1, 1, 1.0, 0.5, 0.5)
    m = S.metrics(gt, det, 0.5)                              # strict on both sides
    assert (m["n_t"], m["n_f"]) == (0, 1)
    assert S.iou((0, 0, 0, 0), (0, 0, 0, 0)) == 1.0
    assert S.iou((0, 0, 1, 1), (1, 1, 2, 2)) == pytest.approx(1 / 7)
    m = S.metrics(gt, [], 0.4)
    assert m["n_t"] == 0 and np.isnan(m["p_fa"])


def test_scene_generator_places_blocks_at_their_snr():
    sc = SS.make_scene(3, "sparse_wifi", T=400, F=512)
    X = np.fft.fft(sc.x.astype(np.complex128), axis=1)[:, (np.arange(512) - 256) % 512]
    P = np.abs(X) ** 2
    inside = np.zeros(P.shape, bool)
    for (t0, f0, t1, f1), snr in zip(sc.boxes, sc.snr_db):
        inside[t0:t1 + 1, f0:f1 + 1] = True
        got = P[t0:t1 + 1, f0:f1 + 1].mean() / 512
        assert got == pytest.approx(1 + 10 ** (snr / 10), rel=0.1)
    assert P[~inside].mean() / 512 == pytest.approx(1.0, rel=0.02)


def test_pipeline_finds_the_blocks():
    cfg = S.SenseConfig(F=512, T=400)
    sc = SS.make_scene(11, "sparse_wifi", T=400, F=512)
    out = S.sense(sc.x, cfg)
    m = S.metrics(sc.boxes, out["boxes"], 0.4)
    assert m["p_d"] >= 0.75 and m["mean_iou"] > 0.5, m
