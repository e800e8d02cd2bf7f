"""Error metrics used by the GPU-vs-oracle parity tests.

Tolerance readings (how the stated accuracy targets are made precise):
  * EVM relative:  sqrt(sum |xt - xt_ref|^2 / sum |xt_ref|^2) over subcarriers
    whose exact condition number kappa_2(A) <= 1e3 and that are not erased;
    bound 1e-4 for the FP32 path.
  * LLR relative:  |llr - llr_ref| / max(|llr_ref|, 0.01 RMS(llr_ref)),
    maximum over all LLRs; bound 1e-3.
  * hard bits:     identical wherever |llr_ref| > tau, tau = 1e-5 RMS(llr_ref)
    (plain FP32); the count inside the guard band is reported.
"""
import numpy as np


def rel_rms(got, ref):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.sqrt(np.sum(np.abs(got - ref) ** 2) / max(np.sum(np.abs(ref) ** 2), 1e-300)))


def evm_rel(xt, xt_ref, good_sc):
    """xt: [..., n_sc]; good_sc: boolean [n_sc] of subcarriers to include."""
    a = np.asarray(xt)[..., good_sc]
    b = np.asarray(xt_ref)[..., good_sc]
    return rel_rms(a, b)


def llr_rel(llr, llr_ref):
    llr = np.asarray(llr, dtype=np.float64)
    ref = np.asarray(llr_ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(ref ** 2)))
    den = np.maximum(np.abs(ref), 0.01 * rms)
    return float(np.max(np.abs(llr - ref) / den))


def hard_bits_outside_guard(llr, llr_ref, rel_tau=1e-5):
    """Returns (n_mismatch_outside_band, n_inside_band)."""
    llr = np.asarray(llr, dtype=np.float64)
    ref = np.asarray(llr_ref, dtype=np.float64)
    tau = rel_tau * float(np.sqrt(np.mean(ref ** 2)))
    outside = np.abs(ref) > tau
    mism = ((llr < 0) != (ref < 0)) & outside
    return int(np.sum(mism)), int(np.sum(~outside))


def elem_rel(got, ref, floor=0.01):
    """Element-wise relative error of a real or complex array,
    max |got - ref| / max(|ref|, floor * RMS(|ref|)): the LLR metric applied
    to gradients, so that one wrong element fails where a norm would not."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    if ref.size == 0:
        return 0.0
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    den = np.maximum(np.abs(ref), floor * rms)
    return float(np.max(np.abs(got - ref) / np.maximum(den, 1e-300)))
