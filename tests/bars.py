"""Parity bars shared by the GPU tests.

FP32 sums (FP32, BF16 and FP16 storage) are compared with the FP64 oracle
evaluated on the *same stored values* (the oracle's emulation of the storage
rounding), so the only difference left is the kernel's FP32 arithmetic:

* values: RMS of the difference <= 1e-6 and its maximum <= 1e-5, both
  relative to the RMS of the oracle's values;
* gradients: the same two bars relative to the RMS of the oracle's gradient.

These hold for every kernel the library builds (Lagrange and splines up to
C3 at I = 8): the kernels evaluate their weight polynomials in powers of
t - 1/2, which keeps Horner's rule well conditioned, and form the FP32
gradient sums from node values taken relative to the particle's own cell
node.
"""
import numpy as np

TIGHT_RMS = 1e-6
TIGHT_MAX = 1e-5


def rel_errors(gpu, ref):
    """(relative RMS, relative max) of gpu - ref against rms(ref)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = float(np.sqrt(np.mean(ref * ref)))
    d = gpu - ref
    return float(np.sqrt(np.mean(d * d)) / scale), float(np.max(np.abs(d)) / scale)


def check_f32(gpu, ref, what=""):
    """Assert the FP32 parity bar; returns (rel RMS, rel max) for reporting."""
    r, m = rel_errors(gpu, ref)
    assert r <= TIGHT_RMS, f"{what}: rel rms {r:.3e} > {TIGHT_RMS:.1e}"
    assert m <= TIGHT_MAX, f"{what}: rel max {m:.3e} > {TIGHT_MAX:.1e}"
    return r, m
