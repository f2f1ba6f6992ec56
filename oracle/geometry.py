"""Steps 1-3 of the interpolation algorithm and particle binning (oracle).

Test infrastructure only.  Follows Sec. 2.2 (enumerated interpolation steps:
wrap X modulo 2*pi, find the grid cell, form the in-cell offset) and
Sec. 3.3.1 "Ordering the particles locally" (particles stored contiguously per
group, in increasing x3 order, with an ``offset`` array of size groups+1 whose
last entry is the particle count).

Readings (the paper fixes no floating-point sequence):

* L = fl64(2*pi); invd = fl64(N / L) by one IEEE division.
* Per axis, in binary64 with round-to-nearest-even and no fused operations:
      q = floor(x / L);  y = x - fl(L*q)
      if y < 0:  y = y + L
      if y >= L: y = 0
      s = y * invd;  c = floor(s);  t = s - c      (t is exact)
      if c == N: c = 0, t = 0
  "closest grid cell" is read as the cell whose lower node is floor(Xtilde/delta),
  and t = xbar/delta is formed as s - c (equal to it in exact arithmetic).
* The bin of a particle: the (x1, x2) plane is cut into tile columns of
  T x T cells (ntx = ceil(N/T) per axis), each column into windows of W cell
  layers along x3 (nw = ceil(N/W)); bins are ordered column by column (x2 tile
  slowest) and along x3 within a column, i.e. the paper's x3-slice order
  applied inside each column:
      key = ((c2//T)*ntx + c1//T)*nw + c3//W.
* The particle order is the stable sort of keys (ties keep their current order),
  and offsets[b] = number of particles with key < b, offsets[n_bins] = Np.
"""
from __future__ import annotations

import math

import numpy as np

L = 2.0 * math.pi  # fl64(2*pi) = 6.283185307179586


def inv_delta(N: int) -> float:
    """invd = fl64(N / L)."""
    return float(np.float64(N) / np.float64(L))


def wrap(x: np.ndarray) -> np.ndarray:
    """Xtilde = X mod 2*pi in [0, L), by the fixed binary64 sequence above."""
    x = np.asarray(x, dtype=np.float64)
    q = np.floor(np.divide(x, L))
    y = np.subtract(x, np.multiply(L, q))
    y = np.where(y < 0.0, np.add(y, L), y)
    y = np.where(y >= L, 0.0, y)
    return y


def cell_and_offset(x: np.ndarray, N: int):
    """Cell index c (int64) and in-cell offset t = xbar/delta in [0,1) per entry.

    ``x`` may have any shape; every entry is treated as one coordinate.
    """
    y = wrap(x)
    s = np.multiply(y, inv_delta(N))
    c = np.floor(s)
    t = np.subtract(s, c)
    c = c.astype(np.int64)
    top = c >= N
    c = np.where(top, 0, c)
    t = np.where(top, 0.0, t)
    return c, t


def cell_and_offset_scalar(x: float, N: int):
    """Pure-Python version of the same sequence for hand-listed edge cases."""
    q = math.floor(x / L)
    y = x - L * q
    if y < 0.0:
        y = y + L
    if y >= L:
        y = 0.0
    s = y * inv_delta(N)
    c = math.floor(s)
    t = s - c
    if c >= N:
        c, t = 0, 0.0
    return int(c), float(t)


def n_bins(N: int, T: int, W: int) -> int:
    ntx = -(-N // T)
    return ntx * ntx * (-(-N // W))


def bin_keys(X: np.ndarray, N: int, T: int, W: int) -> np.ndarray:
    """Bin key per particle for positions X[Np][3] (x1, x2, x3)."""
    c, _ = cell_and_offset(np.asarray(X, dtype=np.float64), N)
    ntx = -(-N // T)
    nw = -(-N // W)
    return (((c[:, 1] // T) * ntx + c[:, 0] // T) * nw + c[:, 2] // W).astype(np.int64)


def stable_order(keys: np.ndarray) -> np.ndarray:
    """perm with keys[perm] sorted, ties in their current order."""
    return np.argsort(keys, kind="stable")


def offsets_from_keys(keys: np.ndarray, n_bins: int) -> np.ndarray:
    """offsets[b] = #{key < b}, size n_bins+1, last entry = number of particles."""
    counts = np.bincount(np.asarray(keys, dtype=np.int64), minlength=n_bins)
    off = np.zeros(n_bins + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def naive_stable_order(keys) -> list:
    """Insertion-order bucket sort written out in plain Python (tiny inputs)."""
    buckets = {}
    for i, k in enumerate(keys):
        buckets.setdefault(int(k), []).append(i)
    out = []
    for k in sorted(buckets):
        out.extend(buckets[k])
    return out
