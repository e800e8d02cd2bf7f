"""Seeded synthetic spectrum-sensing captures: complex64 I/Q with energy
blocks at known time-frequency boxes.

A capture is T consecutive non-overlapping F-sample segments.  Noise is
CN(0, 1) per sample.  Each energy block (t0, f0, t1, f1), inclusive, in TF
plot coordinates (row = segment, column c = FFT bin (c - F/2) mod F, i.e.
the centred spectrum) is band-limited Gaussian signal drawn in the frequency
domain: every bin of the block's columns in each of its rows gets CN(0,
F * 10^(SNR/10)), and the rows are brought to time samples by numpy's
inverse FFT, so the per-pixel SNR of the block is SNR.  This module draws
inputs only; it holds none of the sensing pipeline's arithmetic.

The scenario parameters stand in for the paper's BLE and Wi-Fi (OFDM and
DSSS) captures at 100 MS/s with F = 1024 (bins of about 97.7 kHz, rows of
10.24 us): BLE blocks 2 MHz wide (20 bins) and 10..200 rows long at 15 dB,
OFDM Wi-Fi 20 MHz (205 bins), 20..200 rows at 20 dB, DSSS Wi-Fi 22 MHz
(225 bins), 20..200 rows at 14 dB.
"""
from __future__ import annotations

import dataclasses

import numpy as np

KINDS = {                 # width in bins at F = 1024, rows (min, max), SNR dB
    "ble": (20, (10, 200), 15.0),
    "ofdm": (205, (20, 200), 20.0),
    "dsss": (225, (20, 200), 14.0),
}

SCENARIOS = {             # kinds drawn, number of blocks
    "sparse_ble": (("ble",), 8),
    "dense_ble": (("ble",), 30),
    "sparse_wifi": (("ofdm", "dsss"), 4),
    "dense_wifi": (("ofdm", "dsss"), 10),
    "mixed": (("ble", "ofdm", "dsss"), 16),
}

GAP = 4                   # minimum spacing between blocks, pixels, both axes


@dataclasses.dataclass
class Scene:
    x: np.ndarray         # complex64 [T][F] time samples, row t = segment t
    boxes: np.ndarray     # int32 [n][4] (t0, f0, t1, f1) inclusive
    snr_db: np.ndarray    # float64 [n]
    T: int
    F: int


def _overlaps(b, placed):
    t0, f0, t1, f1 = b
    for (s0, g0, s1, g1) in placed:
        if t0 <= s1 + GAP and s0 <= t1 + GAP and f0 <= g1 + GAP and g0 <= f1 + GAP:
            return True
    return False


def make_scene(seed: int, scenario: str = "mixed", T: int = 2000, F: int = 1024,
               snr_offset_db: float = 0.0) -> Scene:
    kinds, n_blocks = SCENARIOS[scenario]
    rng = np.random.default_rng([7, seed, len(scenario), T, F])
    placed, snrs = [], []
    scale = F / 1024.0
    for _ in range(n_blocks):
        kind = kinds[rng.integers(len(kinds))]
        w, (lmin, lmax), snr = KINDS[kind]
        w = max(2, int(round(w * scale)))
        for _attempt in range(200):
            L = int(rng.integers(lmin, min(lmax, T - 2) + 1))
            t0 = int(rng.integers(0, T - L + 1))
            f0 = int(rng.integers(0, F - w + 1))
            b = (t0, f0, t0 + L - 1, f0 + w - 1)
            if not _overlaps(b, placed):
                placed.append(b)
                snrs.append(snr + snr_offset_db)
                break
    noise = (rng.standard_normal((T, F)) + 1j * rng.standard_normal((T, F))) * np.sqrt(0.5)
    Xs = np.zeros((T, F), dtype=np.complex128)
    cols = np.arange(F)
    bins = (cols - F // 2) % F
    for (t0, f0, t1, f1), snr in zip(placed, snrs):
        p = F * 10.0 ** (snr / 10.0)
        shp = (t1 - t0 + 1, f1 - f0 + 1)
        v = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * np.sqrt(p / 2)
        Xs[t0:t1 + 1, bins[f0:f1 + 1]] += v
    x = noise + np.fft.ifft(Xs, axis=1)
    boxes = np.array(placed, dtype=np.int32).reshape(-1, 4)
    return Scene(x.astype(np.complex64), boxes, np.array(snrs), T, F)


def make_scenes(seeds, scenario="mixed", T=2000, F=1024):
    return [make_scene(s, scenario, T, F) for s in seeds]
