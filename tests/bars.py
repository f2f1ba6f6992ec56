"""Parity bars shared by the GPU tests.

FP32 sums (FP32, BF16 and FP16 storage) are compared with the FP64 oracle
evaluated on the *same stored values* (the oracle's emulation of the storage
rounding), so the only difference left is the kernel's FP32 arithmetic:

* values: RMS of the difference <= 1e-6 and its maximum <= 1e-5, both
  relative to the RMS of the oracle's values;
* gradients: the same two bars relative to the RMS of the oracle's gradient.

The C3 spline (I = 8, m = 3) is the one documented exception: its polynomial
coefficients are several times larger than those of the other kernels, so
every rounding of its Horner weights and sums is larger too.  For it the
per-element bound 64 * 2^-24 * A applies, with A the oracle's absolute sum
(every field value by its absolute value and every weight by the sum of the
absolute values of its polynomial's terms, sum_p |c_p| t^p), which covers the
first-order rounding of Horner steps and FP32 sums of depth <= 20.
"""
import numpy as np

TIGHT_RMS = 1e-6
TIGHT_MAX = 1e-5
F32_BOUND = 64 * 2.0 ** -24


def rel_errors(gpu, ref):
    """(relative RMS, relative max) of gpu - ref against rms(ref)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = float(np.sqrt(np.mean(ref * ref)))
    d = gpu - ref
    return float(np.sqrt(np.mean(d * d)) / scale), float(np.max(np.abs(d)) / scale)


def is_c3(fam, I, m):
    return fam == 1 and I == 8 and m == 3


def check_f32(gpu, ref, absum=None, c3=False, what="", scale=1.0):
    """Assert the FP32 parity bar; returns (rel RMS, rel max) for reporting.
    `scale` widens the bars for results that went through a documented extra
    rounding (the 16-bit forms' product with s_a)."""
    r, m = rel_errors(gpu, ref)
    if c3:
        assert absum is not None, "the C3 exception needs the absolute sum"
        ok = bool(np.all(np.abs(np.asarray(gpu, np.float64) - ref) <= F32_BOUND * absum * scale))
        assert ok, f"{what}: outside the C3 per-element bound (rel rms {r:.2e}, max {m:.2e})"
    else:
        assert r <= TIGHT_RMS * scale, f"{what}: rel rms {r:.3e} > {TIGHT_RMS * scale:.1e}"
        assert m <= TIGHT_MAX * scale, f"{what}: rel max {m:.3e} > {TIGHT_MAX * scale:.1e}"
    return r, m
