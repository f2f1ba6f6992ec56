"""Reduced-precision field storage, emulated bit for bit (oracle).

Test infrastructure only.  The paper computes everything in double precision
(Sec. 4.2); storing the field in FP32, BF16 or FP16 with FP32 weights and sums
is a form beside the paper's method.  Readings:

* FP64 and FP32 storage keep the field unscaled (FP32 = round-to-nearest-even
  of the FP64 value, or the FP32 input itself).
* BF16 / FP16 storage scales each component by its root-mean-square over the
  grid: s_a = sqrt(mean(u_a^2)) in FP64, inv_a = fl32(1/s_a), and stores
  RNE_{bf16|f16}(fl32(u_a * inv_a)) where u_a is the FP32 field value.
* Interpolation on the stored field sums in FP32 and multiplies the result by
  fl32(s_a).  The oracle's "tight" reference is the FP64 sum over the stored
  (already rounded) values times fl32(s_a).
"""
from __future__ import annotations

import numpy as np

F64, F32, BF16, F16 = 0, 1, 2, 3


def component_rms(u: np.ndarray) -> np.ndarray:
    """s_a = sqrt(mean over the grid of u_a^2), FP64, for u[..., 3]."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    return np.sqrt(np.mean(u * u, axis=0))


def f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even); returns uint16 bits."""
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def store(u: np.ndarray, storage: int):
    """Return (stored values as FP64 array, fl32(s_a) as FP64 [3]) for a field u[...,3].

    ``u`` holds the caller's field values (FP32 or FP64).
    """
    u = np.asarray(u)
    if storage == F64:
        return u.astype(np.float64), np.ones(3)
    if storage == F32:
        return u.astype(np.float32).astype(np.float64), np.ones(3)
    s = component_rms(u)
    inv32 = (1.0 / s).astype(np.float32)
    scaled = np.multiply(u.astype(np.float32), inv32)          # fl32(u32 * inv32)
    if storage == BF16:
        vals = bf16_bits_to_f64(f32_to_bf16_bits(scaled))
    elif storage == F16:
        vals = scaled.astype(np.float16).astype(np.float64)
    else:
        raise ValueError("unknown storage type")
    return vals, s.astype(np.float32).astype(np.float64)
