"""Seeded frame synthesis for the uplink receiver workloads.

Frame structure (one frame = one slot):
  * n_sym = 14 OFDM symbols; symbol 0 carries comb pilots, symbols 1..13 data.
  * n_sc used subcarriers, contiguous and centred on DC with DC kept:
    used subcarrier i sits on FFT bin (i - n_sc//2) mod n_fft.
  * comb pilots: in symbol 0, used subcarrier i carries user (i mod K)'s
    unit-modulus QPSK pilot p[i]; every other user is silent there.
  * the channel is block-constant over pilot groups of K consecutive
    subcarriers (the trailing n_sc mod K subcarriers join the last group),
    and constant over the 14 symbols.
  * frequency-domain noise variance N0 = 1 per resource element per antenna;
    user u transmits with power P_u = 10^(SNR_u/10), folded into the
    effective channel h[m][u][i] = sqrt(P_u) * H[m][u][i].
  * time samples are numpy-style ifft (1/N) of the grid plus time-domain
    noise CN(0, N0/N), with an optional cyclic prefix, cast to complex64.

Random draws come from ``np.random.default_rng([config, frame, stream])``
so every input can be regenerated from its coordinates.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STREAMS = {"bits": 0, "pilots": 1, "channel": 2, "noise": 3, "snr": 4,
           "shape": 5, "theta": 6}

MODULATION = {2: "QPSK", 4: "16QAM", 6: "64QAM"}


@dataclasses.dataclass(frozen=True)
class Shape:
    M: int             # base-station antennas
    K: int             # users
    n_fft: int         # FFT size (power of two)
    n_sc: int          # used subcarriers
    n_sym: int = 14    # OFDM symbols per frame, symbol 0 = pilots
    cp_len: int = 0    # cyclic-prefix samples per symbol
    qam_bits: int = 2  # bits per QAM symbol (2, 4 or 6)

    @property
    def n_data(self) -> int:
        return self.n_sym - 1

    @property
    def detections(self) -> int:
        """Subcarrier-detections per frame: one per (data symbol, used subcarrier)."""
        return self.n_sc * self.n_data

    @property
    def sym_len(self) -> int:
        return self.cp_len + self.n_fft


@dataclasses.dataclass
class Frame:
    shape: Shape
    x: np.ndarray          # complex64 [M][n_sym][cp+N] received time samples
    pilots: np.ndarray     # complex64 [n_sc]
    bits: np.ndarray       # uint8 [K][D][n_sc][Q] transmitted bits
    symbols: np.ndarray    # complex128 [K][D][n_sc] transmitted unit-energy symbols
    h: np.ndarray          # complex128 [M][K][n_sc] effective channel (power folded in)
    snr_db: np.ndarray     # float64 [K]
    n0: float
    channel: str
    extra: dict = dataclasses.field(default_factory=dict)


# Workload configurations, each named by what it is.
CONFIGS = {
    1: dict(name="8x2 N512 300sc QPSK Rayleigh 20dB",
            shape=Shape(8, 2, 512, 300, 14, 0, 2), channel="rayleigh",
            snr=(20.0, 20.0), frames=1, detector="zf"),
    2: dict(name="64x16 N2048 1200sc 16QAM Rayleigh 10-30dB",
            shape=Shape(64, 16, 2048, 1200, 14, 0, 4), channel="rayleigh",
            snr=(10.0, 30.0), frames=100, detector="zf"),
    3: dict(name="64x16 N4096 3276sc 64QAM Kronecker(0.7,0.3) 25dB",
            shape=Shape(64, 16, 4096, 3276, 14, 0, 6), channel="kronecker",
            snr=(25.0, 25.0), frames=100, detector="zf"),
    4: dict(name="256 uneven frames, Rayleigh 5-30dB",
            shape=None, channel="rayleigh", snr=(5.0, 30.0), frames=256,
            detector="mmse"),
    5: dict(name="64x8 N2048 1200sc 16QAM cascaded(256 phases) 5dB",
            shape=Shape(64, 8, 2048, 1200, 14, 0, 4), channel="cascaded",
            snr=(5.0, 5.0), frames=1, detector="mmse"),
}


def config_shape(cfg: int) -> Shape:
    s = CONFIGS[cfg]["shape"]
    if s is None:
        raise ValueError("config %d draws a shape per frame" % cfg)
    return s


def _rng(cfg: int, frame: int, stream: str) -> np.random.Generator:
    return np.random.default_rng([int(cfg), int(frame), STREAMS[stream]])


def _cn(rng: np.random.Generator, shape, var: float = 1.0) -> np.ndarray:
    """Circularly-symmetric complex normal with the given variance."""
    s = math.sqrt(var / 2.0)
    return s * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def used_bins(n_fft: int, n_sc: int) -> np.ndarray:
    """FFT bin of each used subcarrier: centred block, DC kept."""
    return (np.arange(n_sc) - n_sc // 2) % n_fft


def pilot_user(n_sc: int, K: int) -> np.ndarray:
    """User that owns the comb pilot on each used subcarrier of symbol 0."""
    return np.arange(n_sc) % K


def qam_map(bits: np.ndarray, q: int) -> np.ndarray:
    """Gray square QAM with unit average energy; bits[..., 0] is b0.

    QPSK  (1/sqrt2)  [(1-2b0) + j(1-2b1)]
    16QAM (1/sqrt10) [(1-2b0)(2-(1-2b2)) + j(1-2b1)(2-(1-2b3))]
    64QAM (1/sqrt42) [(1-2b0)(4-(1-2b2)(2-(1-2b4)))
                      + j(1-2b1)(4-(1-2b3)(2-(1-2b5)))]
    """
    b = 1.0 - 2.0 * np.asarray(bits, dtype=np.float64)  # 0 -> +1, 1 -> -1
    if q == 2:
        return (b[..., 0] + 1j * b[..., 1]) / math.sqrt(2.0)
    if q == 4:
        re = b[..., 0] * (2.0 - b[..., 2])
        im = b[..., 1] * (2.0 - b[..., 3])
        return (re + 1j * im) / math.sqrt(10.0)
    if q == 6:
        re = b[..., 0] * (4.0 - b[..., 2] * (2.0 - b[..., 4]))
        im = b[..., 1] * (4.0 - b[..., 3] * (2.0 - b[..., 5]))
        return (re + 1j * im) / math.sqrt(42.0)
    raise ValueError("qam_bits must be 2, 4 or 6")


def _sqrtm_psd(r: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eigh(r)
    return (v * np.sqrt(np.clip(w, 0.0, None))) @ v.conj().T


def _exp_corr(n: int, rho: float) -> np.ndarray:
    idx = np.arange(n)
    return rho ** np.abs(idx[:, None] - idx[None, :])


def _group_of(n_sc: int, K: int) -> np.ndarray:
    G = n_sc // K
    if G < 1:
        raise ValueError("n_sc must be >= K")
    return np.minimum(np.arange(n_sc) // K, G - 1)


def _draw_channel(cfg: int, frame: int, shape: Shape, kind: str):
    """Unit-power channel H[m][u][i] (before the user power) and extras."""
    M, K, n_sc = shape.M, shape.K, shape.n_sc
    rng = _rng(cfg, frame, "channel")
    extra = {}
    if kind == "rayleigh":
        G = n_sc // K
        Hg = _cn(rng, (G, M, K))
        H = Hg[_group_of(n_sc, K)]                 # [n_sc][M][K]
    elif kind == "kronecker":
        G = n_sc // K
        rb = _sqrtm_psd(_exp_corr(M, 0.7))
        ru = _sqrtm_psd(_exp_corr(K, 0.3))
        Hw = _cn(rng, (G, M, K))
        Hg = rb[None] @ Hw @ ru[None]
        H = Hg[_group_of(n_sc, K)]
    elif kind == "cascaded":
        n_el = 256
        Gm = _cn(rng, (M, n_el))
        Fm = _cn(rng, (n_el, K))
        Hd = _cn(rng, (M, K))
        theta = _rng(cfg, frame, "theta").uniform(0.0, 2.0 * math.pi, n_el)
        Hflat = cascaded_channel(theta, Gm, Fm, Hd)
        H = np.broadcast_to(Hflat, (n_sc, M, K))
        extra.update(theta=theta, G=Gm, F=Fm, Hd=Hd)
    else:
        raise ValueError("unknown channel model %r" % kind)
    return np.ascontiguousarray(np.moveaxis(H, 0, -1)), extra   # [M][K][n_sc]


def cascaded_channel(theta, Gm, Fm, Hd):
    """H = (1/sqrt(n_el)) G diag(exp(j theta)) F + 0.1 H_d  (frequency flat)."""
    n_el = Gm.shape[1]
    return (Gm * np.exp(1j * np.asarray(theta))[None, :]) @ Fm / math.sqrt(n_el) + 0.1 * Hd


def synthesize(shape: Shape, h_eff, symbols, pilots, noise_t):
    """Time samples [M][S][cp+N] (complex128) of the grid seen through h_eff."""
    M, K, N, n_sc = shape.M, shape.K, shape.n_fft, shape.n_sc
    S = shape.n_sym
    Y = np.zeros((M, S, n_sc), dtype=np.complex128)
    pu = pilot_user(n_sc, K)
    Y[:, 0, :] = h_eff[:, pu, np.arange(n_sc)] * pilots[None, :]
    for u in range(K):
        Y[:, 1:, :] += h_eff[:, u, None, :] * symbols[None, u]
    grid = np.zeros((M, S, N), dtype=np.complex128)
    grid[..., used_bins(N, n_sc)] = Y
    xt = np.fft.ifft(grid, axis=-1) + noise_t
    if shape.cp_len:
        xt = np.concatenate([xt[..., N - shape.cp_len:], xt], axis=-1)
    return xt


def make_frame(cfg: int, frame: int, shape: Shape | None = None,
               channel: str | None = None, snr: tuple | None = None,
               n0: float = 1.0, keep_noise: bool = False) -> Frame:
    """Draw frame number ``frame`` of workload ``cfg``."""
    c = CONFIGS.get(cfg, CONFIGS[2])
    if shape is None:
        shape = c["shape"] if c["shape"] is not None else draw_batch_shapes(frame + 1, cfg)[frame]
    channel = channel or c["channel"]
    lo, hi = snr if snr is not None else c["snr"]
    M, K, N, n_sc, Q = shape.M, shape.K, shape.n_fft, shape.n_sc, shape.qam_bits
    D, S = shape.n_data, shape.n_sym
    if not (1 <= K <= M and K <= n_sc <= N and N & (N - 1) == 0):
        raise ValueError("inconsistent shape %r" % (shape,))

    bits = _rng(cfg, frame, "bits").integers(0, 2, (K, D, n_sc, Q), dtype=np.uint8)
    symbols = qam_map(bits, Q)
    pr = _rng(cfg, frame, "pilots").integers(0, 2, (n_sc, 2))
    pilots = qam_map(pr, 2)
    snr_db = _rng(cfg, frame, "snr").uniform(lo, hi, K) if hi > lo else np.full(K, float(lo))
    H, extra = _draw_channel(cfg, frame, shape, channel)
    amp = np.sqrt(10.0 ** (snr_db / 10.0))
    h_eff = H * amp[None, :, None]
    noise_t = _cn(_rng(cfg, frame, "noise"), (M, S, N), n0 / N)
    x = synthesize(shape, h_eff, symbols, pilots, noise_t)
    if keep_noise:
        extra["noise_t"] = noise_t
    extra["amp"] = amp
    return Frame(shape=shape, x=x.astype(np.complex64), pilots=pilots.astype(np.complex64),
                 bits=bits, symbols=symbols, h=h_eff, snr_db=snr_db, n0=float(n0),
                 channel=channel, extra=extra)


def make_frames(cfg: int, n: int, start: int = 0, **kw) -> list:
    return [make_frame(cfg, start + f, **kw) for f in range(n)]


def _draw_inputs(args):
    cfg, f, shape = args
    fr = make_frame(cfg, f, shape=shape)
    return fr.x, fr.pilots


def draw_inputs(cfg: int, frames, shapes=None, workers: int = 8) -> list:
    """[(x, pilots)] of the listed frame numbers of workload ``cfg`` (optional
    explicit shapes), drawn in forked worker processes; same values as
    make_frame."""
    import concurrent.futures as cf
    import multiprocessing as mp
    frames = list(frames)
    shapes = list(shapes) if shapes is not None else [None] * len(frames)
    jobs = [(cfg, f, s) for f, s in zip(frames, shapes)]
    if workers <= 1 or len(jobs) <= 1:
        return [_draw_inputs(j) for j in jobs]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_draw_inputs, jobs, chunksize=max(1, len(jobs) // (4 * workers))))


def draw_batch_shapes(n: int, cfg: int = 4) -> list:
    """Uneven frame shapes: M in {8,16,32,64}, K in 1..min(16,M), n_sc in
    [300, 3276], n_fft the next power of two >= 1.2 n_sc, QPSK/16/64-QAM."""
    out = []
    for f in range(n):
        r = _rng(cfg, f, "shape")
        M = int(r.choice([8, 16, 32, 64]))
        K = int(r.integers(1, min(16, M) + 1))
        n_sc = int(r.integers(300, 3277))
        N = 1 << int(math.ceil(math.log2(1.2 * n_sc)))
        Q = int(r.choice([2, 4, 6]))
        out.append(Shape(M, K, N, n_sc, 14, 0, Q))
    return out


def fft_framing(n_fft: int, fs: float, sample_bits: int):
    """Segment framing of a non-overlapping n_fft-point FFT at rate fs.

    Returns (dt, df, rate): time resolution n_fft/fs, frequency resolution
    fs/n_fft, and the FFT-stage rate n_fft*sample_bits/dt in bit/s.
    """
    dt = n_fft / fs
    df = fs / n_fft
    return dt, df, n_fft * sample_bits / dt


def quantize_sc16(x, headroom: float = 2.0):
    """The radio's 16-bit fixed-point I/Q: a power-of-two scale chosen so that
    the largest component times `headroom` fits in int16, each component
    rounded to the nearest integer.  Returns (int16 [..., 2], scale); the
    samples are q * scale."""
    x = np.asarray(x)
    peak = float(max(np.abs(x.real).max(), np.abs(x.imag).max(), 1e-30))
    scale = 2.0 ** np.ceil(np.log2(peak * headroom / 32767.0))
    q = np.stack([np.rint(x.real / scale), np.rint(x.imag / scale)], axis=-1)
    return np.clip(q, -32768, 32767).astype(np.int16), float(scale)
