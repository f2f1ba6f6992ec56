"""Seeded synthetic velocity fields on the periodic grid [0, 2*pi)^3.

Layout of every grid returned here: ``u[x3][x2][x1][a]`` (x1 fastest, the three
components fastest within a node), grid spacing delta = 2*pi/N, node j at j*delta.

* ``fourier_mode_field``: u_a(x) = sum_k A_{a,k} cos(k.x + phi_{a,k}) over integer
  wave vectors 1 <= |k| <= kmax in a half space, A ~ N(0,1), phi ~ U[0, 2*pi),
  numpy ``default_rng(seed)``.  Grid values are the direct FP64 sum; the same
  sum evaluated at arbitrary points (``fourier_mode_eval``) is the exact field.
* ``single_mode_field``: one cosine mode per component, with its exact value and
  gradient, for convergence-order checks.
* ``spectral_field``: solenoidal Gaussian random-phase field
      u^(k) = sqrt(E(|k|) / (4 pi |k|^2)) (1 - k k^T/|k|^2) xi(k),
  xi complex standard normal, E(k) = k^(-5/3) for 1 <= k <= kc and
  k^(-5/3) exp(-(k - kc)/(0.1 kc)) above, modes with any |k_j| >= N/2 removed,
  transformed with an inverse real FFT and scaled so that the mean over grid
  and components of u_a^2 is 1.  Built with torch on the requested device
  (the FFT is input synthesis only).
* ``spectrum_modes``: the same kind of random solenoidal modes as a half
  spectrum ``spec[k2][k3][k1][a]`` (complex128, shape (N, N, N//2+1, 3),
  directions 2 and 3 transposed as in a slab-decomposed solver's Fourier
  array), unscaled, Hermitian on the k1 = 0 and k1 = N/2 planes: each mode
  and its partner at (-k2, -k3) are set to (a + conj b)/2 and its conjugate,
  self-conjugate modes to their real part.  Modes with an index N/2 are zero
  unless ``nyquist`` (then random, made Hermitian the same way).
* ``spectrum_modes_torch``: the same construction as ``spectrum_modes`` with
  torch on the requested device (its own random stream), for full-size grids.
* ``sparse_spectrum``: a few random modes with |k_d| <= kmax, as index lists
  (k2 index, k3 index, k1) and amplitudes [n][3], with the conjugate partner
  of every k1 = 0 mode listed too; for full-size grids.
"""
from __future__ import annotations

import math

import numpy as np

L = 2.0 * math.pi


def _half_space_modes(kmax: int) -> np.ndarray:
    ks = []
    r = range(-kmax, kmax + 1)
    for k3 in r:
        for k2 in r:
            for k1 in r:
                n2 = k1 * k1 + k2 * k2 + k3 * k3
                if n2 < 1 or n2 > kmax * kmax:
                    continue
                if k3 > 0 or (k3 == 0 and (k2 > 0 or (k2 == 0 and k1 > 0))):
                    ks.append((k1, k2, k3))
    return np.array(ks, dtype=np.int64)


def fourier_mode_field(N: int, kmax: int = 8, seed: int = 0):
    """Returns (u[N,N,N,3] float64, modes) with modes = dict(k, A, phi)."""
    k = _half_space_modes(kmax)
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((k.shape[0], 3))
    phi = rng.uniform(0.0, L, (k.shape[0], 3))
    modes = {"k": k, "A": A, "phi": phi}
    x = np.arange(N) * (L / N)
    u = np.empty((N, N, N, 3))
    E1 = np.exp(1j * np.outer(k[:, 0], x))      # [M, N]
    E2 = np.exp(1j * np.outer(k[:, 1], x))
    E3 = np.exp(1j * np.outer(k[:, 2], x))
    for a in range(3):
        C = A[:, a] * np.exp(1j * phi[:, a])
        for i3 in range(N):
            T = (C * E3[:, i3])[:, None] * E2       # [M, N(x2)]
            u[i3, :, :, a] = np.real(T.T @ E1)       # [x2, x1]
    return u, modes


def fourier_mode_eval(modes, X: np.ndarray, gradient: bool = False):
    """Exact field (and gradient [P,a,b]) of a Fourier-mode field at X[P,3]."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    k = modes["k"].astype(np.float64)
    ph = X @ k.T                                   # [P, M]
    u = np.empty((X.shape[0], 3))
    g = np.empty((X.shape[0], 3, 3)) if gradient else None
    for a in range(3):
        arg = ph + modes["phi"][:, a]
        u[:, a] = np.cos(arg) @ modes["A"][:, a]
        if gradient:
            s = -np.sin(arg) * modes["A"][:, a]
            g[:, a, :] = s @ k
    return (u, g) if gradient else u


def single_mode_field(N: int, kvec, amp=(1.0, 0.7, -0.4), phase=(0.3, 1.1, 2.0)):
    """Grid of u_a = amp_a cos(k.x + phase_a) and its exact evaluator."""
    kvec = np.asarray(kvec, dtype=np.float64)
    x = np.arange(N) * (L / N)
    X3, X2, X1 = np.meshgrid(x, x, x, indexing="ij")
    arg = kvec[0] * X1 + kvec[1] * X2 + kvec[2] * X3
    u = np.stack([amp[a] * np.cos(arg + phase[a]) for a in range(3)], axis=-1)

    def exact(X, gradient=False):
        X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
        ar = X @ kvec
        val = np.stack([amp[a] * np.cos(ar + phase[a]) for a in range(3)], axis=-1)
        if not gradient:
            return val
        g = np.stack([-amp[a] * np.sin(ar + phase[a])[:, None] * kvec[None, :]
                      for a in range(3)], axis=1)
        return val, g

    return u, exact


def spectral_field(N: int, kc: float, seed: int, device="cpu", dtype=None):
    """Solenoidal random-phase field as a torch tensor [N,N,N,3] (see module doc)."""
    import torch
    if dtype is None:
        dtype = torch.float32
    cdtype = torch.complex128 if dtype == torch.float64 else torch.complex64
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    kf = torch.fft.fftfreq(N, d=1.0 / N, device=device, dtype=dtype)
    kr = torch.fft.rfftfreq(N, d=1.0 / N, device=device, dtype=dtype)
    K3 = kf.view(N, 1, 1)
    K2 = kf.view(1, N, 1)
    K1 = kr.view(1, 1, -1)
    kk = torch.sqrt(K1 * K1 + K2 * K2 + K3 * K3)
    kk_safe = torch.where(kk > 0, kk, torch.ones_like(kk))
    E = kk_safe ** (-5.0 / 3.0)
    E = torch.where(kk > kc, E * torch.exp(-(kk - kc) / (0.1 * kc)), E)
    keep = (kk >= 1) & (K1.abs() < N / 2) & (K2.abs() < N / 2) & (K3.abs() < N / 2)
    amp = torch.where(keep, torch.sqrt(E / (4.0 * math.pi * kk_safe * kk_safe)),
                      torch.zeros_like(E))
    del E
    shape = (N, N, N // 2 + 1)

    def cnormal():
        re = torch.randn(shape, generator=gen, device=device, dtype=dtype)
        im = torch.randn(shape, generator=gen, device=device, dtype=dtype)
        return torch.complex(re, im) * (1.0 / math.sqrt(2.0))

    xi = [cnormal() for _ in range(3)]
    kdot = (K1 * xi[0] + K2 * xi[1] + K3 * xi[2]) / kk_safe
    Ks = (K1, K2, K3)
    out = torch.empty((N, N, N, 3), device=device, dtype=dtype)
    for a in range(3):
        uh = (xi[a] - (Ks[a] / kk_safe) * kdot) * amp
        xi[a] = None
        out[..., a] = torch.fft.irfftn(uh.to(cdtype), s=(N, N, N), dim=(0, 1, 2))
        del uh
    del kdot, xi
    ms = torch.mean(out.to(torch.float64) ** 2) if N <= 256 else _chunked_ms(out)
    out *= (1.0 / math.sqrt(float(ms)))
    return out


def _chunked_ms(u):
    import torch
    acc = 0.0
    for i in range(0, u.shape[0], 64):
        acc += float(torch.sum(u[i:i + 64].to(torch.float64) ** 2))
    return acc / u.numel()


def _hermitian_planes(spec: np.ndarray) -> np.ndarray:
    N = spec.shape[0]
    r = (-np.arange(N)) % N
    for k1 in sorted({0, N // 2}):
        P = spec[:, :, k1, :]
        partner = np.conj(P[r][:, r])
        spec[:, :, k1, :] = (P + partner) / 2.0
    return spec


def spectrum_modes(N: int, kc: float, seed: int, nyquist: bool = False) -> np.ndarray:
    """Random solenoidal half spectrum spec[k2][k3][k1][a] (see module doc)."""
    if N % 2:
        raise ValueError("N must be even")
    H = N // 2 + 1
    rng = np.random.default_rng(seed)
    kf = np.fft.fftfreq(N, d=1.0 / N)
    K2 = kf[:, None, None]
    K3 = kf[None, :, None]
    K1 = np.arange(H, dtype=np.float64)[None, None, :]
    kk = np.sqrt(K1 * K1 + K2 * K2 + K3 * K3)
    kk_safe = np.where(kk > 0, kk, 1.0)
    E = kk_safe ** (-5.0 / 3.0)
    E = np.where(kk > kc, E * np.exp(-(kk - kc) / (0.1 * kc)), E)
    amp = np.where(kk >= 1, np.sqrt(E / (4.0 * math.pi * kk_safe * kk_safe)), 0.0)
    xi = (rng.standard_normal((N, N, H, 3)) + 1j * rng.standard_normal((N, N, H, 3))) / math.sqrt(2.0)
    Ks = (K1, K2, K3)
    kdot = sum(Ks[a] * xi[..., a] for a in range(3)) / kk_safe
    spec = np.empty((N, N, H, 3), dtype=np.complex128)
    for a in range(3):
        spec[..., a] = (xi[..., a] - (Ks[a] / kk_safe) * kdot) * amp
    idx = np.arange(N)
    nyq = (idx[:, None, None] == N // 2) | (idx[None, :, None] == N // 2) | (np.arange(H)[None, None, :] == N // 2)
    if nyquist:
        spec[nyq] = (rng.standard_normal((int(nyq.sum()), 3))
                     + 1j * rng.standard_normal((int(nyq.sum()), 3))) * float(np.mean(amp[amp > 0]))
    else:
        spec[nyq] = 0.0
    return _hermitian_planes(spec)


def sparse_spectrum(N: int, n_modes: int, kmax: int, seed: int):
    """(k2 index, k3 index, k1, amp[n][3]) for n_modes random modes plus the
    conjugate partners of the k1 = 0 ones (see module doc)."""
    rng = np.random.default_rng(seed)
    chosen = {}
    while len(chosen) < n_modes:
        k1 = int(rng.integers(0, kmax + 1))
        k2 = int(rng.integers(-kmax, kmax + 1))
        k3 = int(rng.integers(-kmax, kmax + 1))
        key = (k2 % N, k3 % N, k1)
        pkey = ((-k2) % N, (-k3) % N, k1)
        if key in chosen or (k1 == 0 and pkey in chosen):
            continue
        a = (rng.standard_normal(3) + 1j * rng.standard_normal(3)) / math.sqrt(2.0)
        if k1 == 0:
            if key == pkey:
                a = a.real + 0j
            else:
                chosen[pkey] = np.conj(a)
        chosen[key] = a
    keys = sorted(chosen)
    k2i = np.array([k[0] for k in keys], dtype=np.int64)
    k3i = np.array([k[1] for k in keys], dtype=np.int64)
    k1 = np.array([k[2] for k in keys], dtype=np.int64)
    amp = np.array([chosen[k] for k in keys], dtype=np.complex128)
    return k2i, k3i, k1, amp


def spectrum_modes_torch(N: int, kc: float, seed: int, device="cpu", dtype=None):
    """Random solenoidal half spectrum spec[k2][k3][k1][a] as a torch complex
    tensor on `device` (complex128 unless dtype=torch.complex64), Hermitian on
    the k1 = 0 and N/2 planes, no modes with an index N/2 (see module doc)."""
    import torch
    if N % 2:
        raise ValueError("N must be even")
    cdt = torch.complex128 if dtype is None else dtype
    rdt = torch.float64 if cdt == torch.complex128 else torch.float32
    H = N // 2 + 1
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    kf = torch.fft.fftfreq(N, d=1.0 / N, device=device, dtype=rdt)
    K2 = kf.view(N, 1, 1)
    K3 = kf.view(1, N, 1)
    K1 = torch.arange(H, device=device, dtype=rdt).view(1, 1, H)
    kk = torch.sqrt(K1 * K1 + K2 * K2 + K3 * K3)
    kk_safe = torch.where(kk > 0, kk, torch.ones_like(kk))
    E = kk_safe ** (-5.0 / 3.0)
    E = torch.where(kk > kc, E * torch.exp(-(kk - kc) / (0.1 * kc)), E)
    keep = (kk >= 1) & (K1.abs() < N / 2) & (K2.abs() < N / 2) & (K3.abs() < N / 2)
    amp = torch.where(keep, torch.sqrt(E / (4.0 * math.pi * kk_safe * kk_safe)), torch.zeros_like(E))
    del E, kk, keep
    spec = torch.empty((N, N, H, 3), dtype=cdt, device=device)
    for a in range(3):
        re = torch.randn((N, N, H), generator=gen, device=device, dtype=rdt)
        im = torch.randn((N, N, H), generator=gen, device=device, dtype=rdt)
        spec[..., a] = torch.complex(re, im) * (1.0 / math.sqrt(2.0))
        del re, im
    Ks = (K1, K2, K3)
    kdot = (K1 * spec[..., 0] + K2 * spec[..., 1] + K3 * spec[..., 2]) / kk_safe
    for a in range(3):
        spec[..., a] = (spec[..., a] - (Ks[a] / kk_safe) * kdot) * amp
    del kdot, amp
    r = (-torch.arange(N, device=device)) % N
    for k1 in sorted({0, N // 2}):
        P = spec[:, :, k1, :].clone()
        spec[:, :, k1, :] = (P + torch.conj(P[r][:, r])) / 2.0
    return spec
