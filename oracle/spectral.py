"""Velocity on the grid from the spectral state (oracle).

Test infrastructure only.  Follows Sec. 2.1 (the two representations of a
field: values on the N^3 grid with spacing delta = 2 pi / N, and, by the
Hermitian symmetry of a real field, N x N x (N/2+1) complex Fourier mode
amplitudes; the Biot-Savart law u^(k) = i k x w^(k) / k^2 giving the velocity
from the vorticity) and Sec. 3.2 (the Fourier-space array is distributed along
k2 where the grid is distributed along x3: directions 2 and 3 are transposed
between the representations).  Sec. 4.2 names the step: the extra inverse
transform that particle tracking needs ("IFT for PT").

Layouts:
* spectrum ``spec[k2][k3][k1][a]``, complex, shape (N, N, N//2+1, 3); index j
  on the k2 and k3 axes is the wave number j for j <= N/2 and j - N above;
  k1 = 0 .. N/2.
* grid ``u[x3][x2][x1][a]``, node j at j * delta (as everywhere in the oracle).

Readings where the paper is silent:
* amplitudes: u_a(x) = sum over all wave vectors k of u^_a(k) exp(i k.x), the
  Fourier series of the mode amplitudes (no 1/N^3 in the inverse transform);
  the modes with k1 < 0 are the complex conjugates u^(-k) = conj u^(k).
* Biot-Savart: u^(0) = 0, and u^ = 0 on every mode with an index equal to N/2
  (no signed wave number there, and the derivative of such a mode has no real
  representation on the grid).

Functions:
* ``velocity_modes``  -- u^ in grid order [a][k3][k2][k1] (Biot-Savart for a
  vorticity spectrum).
* ``grid_field``      -- the grid values by numpy's inverse real FFT (a library
  primitive), FP64.
* ``series_literal``  -- the series term by term at every node, with the full
  spectrum built by the conjugation rule (explicit loops; tiny N only).
* ``series_sparse``   -- the series at given nodes summed over stored modes
  given as a list, weight 1 on the k1 = 0 and k1 = N/2 planes (their
  conjugate partners are stored in the same plane) and 2 elsewhere; for
  sampled nodes of sparse spectra at any N (``series_at``: the same over the
  non-zero modes of a whole spectrum).
* ``absolute_sum``    -- A_a = that weighted sum of |u^_a(k)|, a bound on
  |u_a| and the scale of the transform's rounding error.
"""
from __future__ import annotations

import numpy as np

VELOCITY, VORTICITY = 0, 1


def signed(j: np.ndarray, N: int) -> np.ndarray:
    """Wave number of FFT-order index j on an axis of N points."""
    j = np.asarray(j, dtype=np.int64)
    return np.where(j <= N // 2, j, j - N)


def velocity_modes(spec: np.ndarray, kind: int = VELOCITY) -> np.ndarray:
    """u^[a][k3][k2][k1] (complex128) from spec[k2][k3][k1][a]."""
    spec = np.asarray(spec, dtype=np.complex128)
    N = spec.shape[0]
    H = N // 2 + 1
    if spec.shape != (N, N, H, 3):
        raise ValueError("spectrum must have shape (N, N, N//2+1, 3)")
    w = np.transpose(spec, (3, 1, 0, 2))  # [a][k3][k2][k1]
    if kind == VELOCITY:
        return w.copy()
    if kind != VORTICITY:
        raise ValueError("kind must be VELOCITY or VORTICITY")
    j = np.arange(N)
    k3 = signed(j, N).astype(np.float64)[:, None, None]
    k2 = signed(j, N).astype(np.float64)[None, :, None]
    k1 = np.arange(H, dtype=np.float64)[None, None, :]
    ksq = k1 * k1 + k2 * k2 + k3 * k3
    nyq = (j[:, None, None] == N // 2) | (j[None, :, None] == N // 2) | (np.arange(H)[None, None, :] == N // 2)
    zero = nyq | (ksq == 0.0)
    # k x w with real k, then multiplied by i / |k|^2
    c = np.stack([k2 * w[2] - k3 * w[1], k3 * w[0] - k1 * w[2], k1 * w[1] - k2 * w[0]])
    safe = np.where(zero, 1.0, ksq)
    u = 1j * c / safe
    u[:, zero] = 0.0
    return u


def grid_field(spec: np.ndarray, kind: int = VELOCITY) -> np.ndarray:
    """u[x3][x2][x1][a] in FP64: numpy's inverse real FFT without normalisation."""
    uh = velocity_modes(spec, kind)
    N = uh.shape[1]
    out = np.empty((N, N, N, 3))
    for a in range(3):
        out[..., a] = np.fft.irfftn(uh[a], s=(N, N, N), axes=(0, 1, 2), norm="forward")
    return out


def full_spectrum(uh_a: np.ndarray) -> np.ndarray:
    """One component's N^3 spectrum [k3][k2][k1] from the stored half: index
    k1 > N/2 holds conj of the stored mode at (N - k1, -k2, -k3) mod N."""
    N = uh_a.shape[0]
    H = N // 2 + 1
    full = np.zeros((N, N, N), dtype=np.complex128)
    for i3 in range(N):
        for i2 in range(N):
            for i1 in range(N):
                if i1 < H:
                    full[i3, i2, i1] = uh_a[i3, i2, i1]
                else:
                    full[i3, i2, i1] = np.conj(uh_a[(N - i3) % N, (N - i2) % N, N - i1])
    return full


def series_literal(spec: np.ndarray, kind: int = VELOCITY) -> np.ndarray:
    """(u[x3][x2][x1][a], largest |imaginary part|): every node summed over
    all N^3 modes of the full spectrum times exp(2 pi i (k.j) / N); the real
    part is u, the imaginary part of a Hermitian spectrum's series vanishes
    up to rounding."""
    uh = velocity_modes(spec, kind)
    N = uh.shape[1]
    out = np.empty((N, N, N, 3))
    imag_max = 0.0
    for a in range(3):
        full = full_spectrum(uh[a])
        for j3 in range(N):
            for j2 in range(N):
                for j1 in range(N):
                    s = 0.0 + 0.0j
                    for i3 in range(N):
                        for i2 in range(N):
                            for i1 in range(N):
                                ph = 2.0 * np.pi * ((i1 * j1 + i2 * j2 + i3 * j3) % N) / N
                                s += full[i3, i2, i1] * complex(np.cos(ph), np.sin(ph))
                    out[j3, j2, j1, a] = s.real
                    imag_max = max(imag_max, abs(s.imag))
    return out, imag_max


def _stored_weight(k1: np.ndarray, N: int) -> np.ndarray:
    return np.where((k1 == 0) | (k1 == N // 2), 1.0, 2.0)


def series_sparse(N: int, k2i: np.ndarray, k3i: np.ndarray, k1: np.ndarray, amp: np.ndarray,
                  nodes: np.ndarray) -> np.ndarray:
    """u at integer nodes[M] = (j1, j2, j3) from stored modes given as index
    lists (k2 index, k3 index, k1) with velocity amplitudes amp[modes][3]:
    the sum of weight * Re(u^(k) exp(i k.x)), x = delta * j."""
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, 3)
    k2i, k3i, k1 = (np.asarray(v, dtype=np.int64) for v in (k2i, k3i, k1))
    amp = np.asarray(amp, dtype=np.complex128).reshape(-1, 3)
    out = np.zeros((nodes.shape[0], 3))
    if k1.size == 0:
        return out
    wgt = _stored_weight(k1, N)
    # phase 2 pi (k.j mod N) / N with integer arithmetic before the division
    kj = (np.outer(nodes[:, 0], k1) + np.outer(nodes[:, 1], k2i) + np.outer(nodes[:, 2], k3i)) % N
    ph = 2.0 * np.pi * kj / N
    e = np.cos(ph) + 1j * np.sin(ph)  # [M, modes]
    for a in range(3):
        out[:, a] = np.real(e * amp[None, :, a]) @ wgt
    return out


def series_at(spec: np.ndarray, nodes: np.ndarray, kind: int = VELOCITY) -> np.ndarray:
    """series_sparse over the non-zero modes of a whole spectrum."""
    uh = velocity_modes(spec, kind)
    N = uh.shape[1]
    i3, i2, i1 = np.nonzero(np.any(uh != 0, axis=0))
    amp = np.stack([uh[a][i3, i2, i1] for a in range(3)], axis=-1)
    return series_sparse(N, i2, i3, i1, amp, nodes)


def absolute_sum(spec: np.ndarray, kind: int = VELOCITY) -> np.ndarray:
    """A_a = sum over stored modes of weight * |u^_a(k)| (weight as series_at)."""
    uh = velocity_modes(spec, kind)
    N = uh.shape[1]
    wgt = _stored_weight(np.arange(N // 2 + 1), N)[None, None, :]
    return np.array([float(np.sum(np.abs(uh[a]) * wgt)) for a in range(3)])
