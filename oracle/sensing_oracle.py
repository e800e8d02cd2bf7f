"""Plain oracle of the paper's spectrum-sensing pipeline (RISE).

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Slow on purpose;
each function follows one step of the paper and can be checked by eye.

Steps (Section IV-B unless noted):
  tf_plot        Section III-A1: magnitudes of non-overlapping F-point FFTs
                 of consecutive segments, one row per segment; Section VI:
                 absolute values, no normalisation.  Column c holds FFT bin
                 (c - F/2) mod F (the centred spectrum).
  psd            the TF plot summed along time, one value per column.
  sg_smooth      Savitzky-Golay smoothing of the PSD (window and order are
                 not given: 21 and 1; edges by mirror reflection).  Orders
                 of 2 and more have negative weights, which ring below the
                 noise level next to strong wide blocks and drag the lowest
                 local minimum under the noise-only columns.
  noise_floor    the lowest local minimum of the smoothed PSD (interior
                 points no larger than both neighbours).
  threshold      theta_PSD = psd_factor * N0 (the rule is not given: 1.1).
  retained       columns whose PSD is not below theta_PSD.
  binarize       per retained column, Otsu's threshold (the argmax of the
                 between-class variance) over a histogram of the column's
                 values (bins not given: 256 over the column's [min, max]);
                 pixels in bins above it are foreground.  The bin of a value
                 and therefore the mask are decided in FP32, the precision
                 the paper processes samples in (Section IV-D); the argmax is
                 exact (integer arithmetic).
  morph          one 3x3 closing, one 3x3 opening, one 1x3 opening along
                 frequency, in the order listed (the last one never changes
                 the mask after a 3x3 opening), all-ones structuring
                 elements; erosion and dilation take the structuring
                 element's pixels inside the plot only.
  boxes          4-connected components found by one raster scan, each
                 component's inclusive (t0, f0, t1, f1), in the order the
                 scan meets them.
  metrics        Section III-A: IoU matrix, N_t, N_f, P_d, P_fa.

Floating point is float64 except where FP32 is stated.  Library primitives:
numpy's FFT, least squares and sums.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class SenseConfig:
    F: int = 1024
    T: int = 2000
    sg_window: int = 21
    sg_order: int = 1
    psd_factor: float = 1.1
    bins: int = 256


# ---------------------------------------------------------------- TF plot
def tf_plot(x, F: int) -> np.ndarray:
    """x: complex [..., T, F] segments -> float64 [..., T, F] magnitudes,
    column c = bin (c - F/2) mod F."""
    X = np.fft.fft(np.asarray(x, dtype=np.complex128), axis=-1)
    cols = (np.arange(F) - F // 2) % F
    return np.abs(X[..., cols])


def psd(tf) -> np.ndarray:
    """Per-column sum over time (rows)."""
    return np.sum(np.asarray(tf, dtype=np.float64), axis=-2)


# ------------------------------------------------------ Savitzky-Golay
def sg_coeffs(window: int, order: int) -> np.ndarray:
    """Weights c[k], k = -h..h, such that sum_k c[k] y[j + k] is the value at
    offset 0 of the least-squares polynomial of degree `order` through the
    window (the first row of the pseudo-inverse of the Vandermonde matrix)."""
    if window % 2 == 0 or window < 3 or order < 0 or order >= window:
        raise ValueError("window must be odd >= 3 and order < window")
    h = window // 2
    k = np.arange(-h, h + 1, dtype=np.float64)
    V = k[:, None] ** np.arange(order + 1)[None, :]          # [window, order+1]
    P = np.linalg.pinv(V)                                    # [order+1, window]
    return P[0]


def mirror_index(j: int, n: int) -> int:
    """Reflection about the end samples (the end sample is not repeated)."""
    while j < 0 or j >= n:
        j = -j if j < 0 else 2 * (n - 1) - j
    return j


def sg_smooth(p, window: int, order: int) -> np.ndarray:
    p = np.asarray(p, dtype=np.float64)
    c = sg_coeffs(window, order)
    h = window // 2
    n = p.shape[-1]
    out = np.zeros_like(p)
    for j in range(n):
        idx = [mirror_index(j + k, n) for k in range(-h, h + 1)]
        out[..., j] = p[..., idx] @ c
    return out


def noise_floor(s) -> float:
    """Lowest local minimum: the smallest s[j], 0 < j < n-1, with
    s[j] <= s[j-1] and s[j] <= s[j+1]."""
    s = np.asarray(s, dtype=np.float64)
    n = s.shape[0]
    best = None
    for j in range(1, n - 1):
        if s[j] <= s[j - 1] and s[j] <= s[j + 1]:
            if best is None or s[j] < best:
                best = s[j]
    return float(s.min()) if best is None else float(best)


# ------------------------------------------------------------- Otsu
def column_bins(v32, bins: int):
    """FP32 histogram bin of every value of one column: bins equal parts of
    [min, max], bin = min(bins - 1, floor((v - min) * (bins / (max - min)))).
    Returns (bin indices, lo, hi); all zero when the column is constant."""
    v = np.asarray(v32, dtype=np.float32)
    lo, hi = np.float32(v.min()), np.float32(v.max())
    if not hi > lo:
        return np.zeros(v.shape, dtype=np.int64), lo, hi
    scale = np.float32(bins) / np.float32(hi - lo)
    b = np.floor((v - lo) * scale).astype(np.int64)
    return np.minimum(b, bins - 1), lo, hi


def otsu_threshold(b, bins: int) -> int:
    """Otsu's threshold bin k (class 0 = bins <= k) maximising the
    between-class variance omega0 omega1 (mu0 - mu1)^2 of the bin indices,
    i.e. (N m0 - M omega0)^2 / (omega0 omega1) with m0 = sum of indices in
    class 0 and M over all; ties go to the smallest k; -1 if no k leaves both
    classes non-empty.  Python integers: exact."""
    h = np.bincount(np.asarray(b, dtype=np.int64), minlength=bins)
    N = int(h.sum())
    M = int(np.dot(np.arange(bins), h))
    best_k, best_num, best_den = -1, 0, 1
    w0 = m0 = 0
    for k in range(bins - 1):
        w0 += int(h[k])
        m0 += k * int(h[k])
        w1 = N - w0
        if w0 == 0 or w1 == 0:
            continue
        num = (N * m0 - M * w0) ** 2
        den = w0 * w1
        if best_k < 0 or num * best_den > best_num * den:
            best_k, best_num, best_den = k, num, den
    return best_k


def binarize(tf32, retained, bins: int):
    """tf32 [T][F] float32, retained bool [F] -> (mask uint8 [T][F], k int [F]
    with -1 for pruned columns and columns without a threshold)."""
    tf32 = np.asarray(tf32, dtype=np.float32)
    T, F = tf32.shape
    mask = np.zeros((T, F), dtype=np.uint8)
    ks = np.full(F, -1, dtype=np.int64)
    for j in range(F):
        if not retained[j]:
            continue
        b, _, _ = column_bins(tf32[:, j], bins)
        k = otsu_threshold(b, bins)
        ks[j] = k
        if k >= 0:
            mask[:, j] = b > k
    return mask, ks


# --------------------------------------------------- morphology
def dilate(a, dt: int, df: int):
    """Max over the (2dt+1) x (2df+1) neighbourhood inside the plot."""
    a = np.asarray(a, dtype=np.uint8)
    T, F = a.shape
    out = np.zeros_like(a)
    p = np.pad(a, ((dt, dt), (df, df)), constant_values=0)
    for i in range(2 * dt + 1):
        for j in range(2 * df + 1):
            out = np.maximum(out, p[i:i + T, j:j + F])
    return out


def erode(a, dt: int, df: int):
    """Min over the neighbourhood inside the plot (outside counts as 1)."""
    a = np.asarray(a, dtype=np.uint8)
    T, F = a.shape
    out = np.ones_like(a)
    p = np.pad(a, ((dt, dt), (df, df)), constant_values=1)
    for i in range(2 * dt + 1):
        for j in range(2 * df + 1):
            out = np.minimum(out, p[i:i + T, j:j + F])
    return out


def morph(mask):
    """3x3 closing, then 3x3 opening, then 1x3 opening along frequency, the
    order the paper lists them in.  The last step never changes the mask: a
    3x3 opening leaves a union of 3x3 squares, which every 1x3 opening
    keeps; it is applied all the same."""
    a = erode(dilate(mask, 1, 1), 1, 1)         # closing
    a = dilate(erode(a, 1, 1), 1, 1)            # opening
    a = dilate(erode(a, 0, 1), 0, 1)            # horizontal opening
    return a


# ------------------------------------------------------- CCL and boxes
def boxes(mask) -> np.ndarray:
    """One raster scan; an unvisited foreground pixel starts a component,
    flood-filled through 4-neighbours.  int32 [n][4] (t0, f0, t1, f1)."""
    m = np.asarray(mask, dtype=bool)
    T, F = m.shape
    seen = np.zeros((T, F), dtype=bool)
    out = []
    for t in range(T):
        row = m[t]
        if not row.any():
            continue
        for f in np.nonzero(row & ~seen[t])[0]:
            if seen[t, f]:
                continue
            t0 = t1 = t
            f0 = f1 = int(f)
            stack = [(t, int(f))]
            seen[t, f] = True
            while stack:
                a, b = stack.pop()
                t0, t1, f0, f1 = min(t0, a), max(t1, a), min(f0, b), max(f1, b)
                for na, nb in ((a - 1, b), (a + 1, b), (a, b - 1), (a, b + 1)):
                    if 0 <= na < T and 0 <= nb < F and m[na, nb] and not seen[na, nb]:
                        seen[na, nb] = True
                        stack.append((na, nb))
            out.append((t0, f0, t1, f1))
    return np.array(out, dtype=np.int32).reshape(-1, 4)


# ------------------------------------------------------------ metrics
def iou(a, b) -> float:
    """Intersection over union of two inclusive pixel boxes."""
    it = min(a[2], b[2]) - max(a[0], b[0]) + 1
    jf = min(a[3], b[3]) - max(a[1], b[1]) + 1
    inter = max(it, 0) * max(jf, 0)
    area = lambda x: (x[2] - x[0] + 1) * (x[3] - x[1] + 1)  # noqa: E731
    return inter / (area(a) + area(b) - inter)


def metrics(gt, det, theta: float) -> dict:
    """Section III-A: I_ij = IoU(B_i, B^_j); N_t counts ground truths whose
    best IoU exceeds theta, N_f detections whose best IoU is below theta;
    P_d = N_t / N_gt, P_fa = N_f / N_d (NaN for an empty denominator);
    mean_iou = the mean over ground truths of their best IoU."""
    gt, det = np.asarray(gt).reshape(-1, 4), np.asarray(det).reshape(-1, 4)
    I = np.zeros((len(gt), len(det)))
    for i in range(len(gt)):
        for j in range(len(det)):
            I[i, j] = iou(gt[i], det[j])
    n_t = int(sum(1 for i in range(len(gt)) if len(det) and I[i].max() > theta))
    n_f = int(sum(1 for j in range(len(det)) if len(gt) == 0 or I[:, j].max() < theta))
    return dict(iou=I, n_t=n_t, n_f=n_f,
                p_d=n_t / len(gt) if len(gt) else float("nan"),
                p_fa=n_f / len(det) if len(det) else float("nan"),
                mean_iou=float(I.max(axis=1).mean()) if len(gt) and len(det) else 0.0)


# ------------------------------------------------------------ pipeline
def sense_from_tf(tf, cfg: SenseConfig) -> dict:
    """Every step after the TF plot; tf is rounded to FP32 for the binarisation."""
    tf = np.asarray(tf)
    p = psd(tf)
    s = sg_smooth(p, cfg.sg_window, cfg.sg_order)
    n0 = noise_floor(s)
    theta = cfg.psd_factor * n0
    retained = p >= theta
    mask, ks = binarize(tf.astype(np.float32), retained, cfg.bins)
    m2 = morph(mask)
    return dict(psd=p, psd_smooth=s, n0=n0, theta=theta, retained=retained, otsu_bin=ks,
                mask=mask, mask_mo=m2, boxes=boxes(m2))


def sense(x, cfg: SenseConfig) -> dict:
    tf = tf_plot(x, cfg.F)
    out = sense_from_tf(tf, cfg)
    out["tf"] = tf
    return out
