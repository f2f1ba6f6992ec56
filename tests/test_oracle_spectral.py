"""Pins of the spectral-state oracle (oracle/spectral.py) against what the
mathematics fixes: the Fourier series summed term by term over the full
spectrum built by the conjugation rule, closed forms of single modes (which
also fix the [k2][k3][k1] order, the sign of the exponent, the weight of the
stored half and the normalisation), Parseval's identity, the bound |u| <= A,
and for the Biot-Savart law the identities div u = 0 and curl u = w checked
through numpy's forward transform of the oracle's grid.

Transform tolerance (FP64): |u - exact| <= 8 log2(N^3) 2^-53 A_a per element,
A_a the absolute sum of the series' terms (an FFT rounds each output through
log2(N^3) butterfly stages whose inputs are bounded by A_a).
"""
import math

import numpy as np
import pytest

from oracle import spectral as sp
from synthetic import fields

EPS = 2.0 ** -53


def fft_tol(N, A):
    return 8.0 * math.log2(N ** 3) * EPS * np.asarray(A)


def nodes_grid(N):
    x = np.arange(N) * (2.0 * math.pi / N)
    X3, X2, X1 = np.meshgrid(x, x, x, indexing="ij")
    return X1, X2, X3


@pytest.mark.parametrize("N,nyq", [(4, True), (6, True), (8, False)])
def test_grid_field_is_the_literal_series(N, nyq):
    spec = fields.spectrum_modes(N, kc=N / 3.0, seed=N, nyquist=nyq)
    lit, imag = sp.series_literal(spec)
    A = sp.absolute_sum(spec)
    tol = fft_tol(N, A)
    assert imag <= float(tol.max())  # the generator's planes are Hermitian
    g = sp.grid_field(spec)
    assert np.all(np.abs(g - lit) <= tol)
    nodes = np.array([[0, 0, 0], [N - 1, 1, 2], [1, N - 1, N // 2], [N // 2, N // 2, N - 1]])
    sa = sp.series_at(spec, nodes)
    assert np.all(np.abs(sa - lit[nodes[:, 2], nodes[:, 1], nodes[:, 0]]) <= tol)


def test_single_modes_closed_forms():
    N = 16
    H = N // 2 + 1
    X1, X2, X3 = nodes_grid(N)
    c = np.array([0.7 - 0.2j, -0.3 + 0.9j, 0.25 + 0.5j])
    # k = (3, -2, 5): stored once, at spec[k2 index][k3 index][k1]
    spec = np.zeros((N, N, H, 3), dtype=np.complex128)
    spec[N - 2, 5, 3, :] = c
    g = sp.grid_field(spec)
    th = 3 * X1 - 2 * X2 + 5 * X3
    for a in range(3):
        exact = 2.0 * (c[a].real * np.cos(th) - c[a].imag * np.sin(th))
        assert np.allclose(g[..., a], exact, rtol=0, atol=1e-13)
    # k = (0, 2, -1) and its partner (0, -2, 1) in the k1 = 0 plane
    spec = np.zeros((N, N, H, 3), dtype=np.complex128)
    spec[2, N - 1, 0, :] = c
    spec[N - 2, 1, 0, :] = np.conj(c)
    g = sp.grid_field(spec)
    th = 2 * X2 - X3
    for a in range(3):
        assert np.allclose(g[..., a], 2.0 * np.real(c[a] * np.exp(1j * th)), rtol=0, atol=1e-13)
    # a mode along x2 only varies along x2 (the k2 axis comes first in spec)
    spec = np.zeros((N, N, H, 3), dtype=np.complex128)
    spec[1, 0, 0, 0] = 0.5
    spec[N - 1, 0, 0, 0] = 0.5
    g = sp.grid_field(spec)
    assert np.allclose(g[..., 0], np.cos(X2), rtol=0, atol=1e-14)
    # the mean, and the self-conjugate mode k1 = N/2: (-1)^j1
    spec = np.zeros((N, N, H, 3), dtype=np.complex128)
    spec[0, 0, 0, :] = [1.5, -2.0, 0.25]
    spec[0, 0, N // 2, 1] = 0.75
    g = sp.grid_field(spec)
    j1 = np.rint(X1 / (2 * math.pi / N)).astype(int)
    assert np.allclose(g[..., 0], 1.5, rtol=0, atol=1e-15)
    assert np.allclose(g[..., 1], -2.0 + 0.75 * (-1.0) ** j1, rtol=0, atol=1e-15)
    assert np.allclose(g[..., 2], 0.25, rtol=0, atol=1e-15)


def test_parseval_and_bound():
    N = 16
    for nyq in (False, True):
        spec = fields.spectrum_modes(N, kc=5.0, seed=4 + nyq, nyquist=nyq)
        g = sp.grid_field(spec)
        uh = sp.velocity_modes(spec)
        w = np.where((np.arange(N // 2 + 1) == 0) | (np.arange(N // 2 + 1) == N // 2), 1.0, 2.0)
        for a in range(3):
            energy = float(np.sum(np.abs(uh[a]) ** 2 * w[None, None, :]))
            assert math.isclose(float(np.mean(g[..., a] ** 2)), energy, rel_tol=1e-12)
        A = sp.absolute_sum(spec)
        assert np.all(np.abs(g).max(axis=(0, 1, 2)) <= A * (1 + 1e-12))


def test_series_sparse_weights():
    """Sparse list form = whole-spectrum form (weights 1 on the k1 = 0, N/2
    planes, 2 elsewhere), and both = the literal series."""
    N = 6
    k2i, k3i, k1, amp = fields.sparse_spectrum(N, 5, 2, seed=3)
    spec = np.zeros((N, N, N // 2 + 1, 3), dtype=np.complex128)
    spec[k2i, k3i, k1] = amp
    lit, imag = sp.series_literal(spec)
    assert imag < 1e-13
    nodes = np.stack(np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij"), -1).reshape(-1, 3)
    s1 = sp.series_sparse(N, k2i, k3i, k1, amp, nodes)
    s2 = sp.series_at(spec, nodes)
    ref = lit[nodes[:, 2], nodes[:, 1], nodes[:, 0]]
    assert np.allclose(s1, ref, rtol=0, atol=1e-13)
    assert np.allclose(s2, ref, rtol=0, atol=1e-13)


def test_biot_savart_single_mode():
    """w = 2 cos(x1) e3 (w^ = 1 on component 3 at k = (1, 0, 0)) has the
    velocity u = (0, 2 sin(x1), 0): curl u = (0, 0, d1 u2) = w."""
    N = 16
    spec = np.zeros((N, N, N // 2 + 1, 3), dtype=np.complex128)
    spec[0, 0, 1, 2] = 1.0
    g = sp.grid_field(spec, sp.VORTICITY)
    X1, _, _ = nodes_grid(N)
    assert np.allclose(g[..., 0], 0.0, atol=1e-15)
    assert np.allclose(g[..., 1], 2.0 * np.sin(X1), rtol=0, atol=1e-14)
    assert np.allclose(g[..., 2], 0.0, atol=1e-15)


def test_biot_savart_curl_and_divergence():
    """For a random solenoidal vorticity without Nyquist modes: the forward
    transform of the oracle's velocity grid has k . u^ = 0, i k x u^ = w^ and
    u^(0) = 0."""
    N = 16
    w = fields.spectrum_modes(N, kc=6.0, seed=9)
    g = sp.grid_field(w, sp.VORTICITY)
    # forward transform (amplitudes), back to spec order [k2][k3][k1][a]
    uh = np.stack([np.fft.rfftn(g[..., a], axes=(0, 1, 2), norm="forward") for a in range(3)], -1)
    uh = np.transpose(uh, (1, 0, 2, 3))
    kf = np.fft.fftfreq(N, d=1.0 / N)
    K2 = kf[:, None, None]
    K3 = kf[None, :, None]
    K1 = np.arange(N // 2 + 1, dtype=np.float64)[None, None, :]
    scale = float(np.abs(w).max())
    div = K1 * uh[..., 0] + K2 * uh[..., 1] + K3 * uh[..., 2]
    assert float(np.abs(div).max()) <= 1e-12 * scale
    curl = 1j * np.stack([K2 * uh[..., 2] - K3 * uh[..., 1],
                          K3 * uh[..., 0] - K1 * uh[..., 2],
                          K1 * uh[..., 1] - K2 * uh[..., 0]], -1)
    assert float(np.abs(curl - w).max()) <= 1e-12 * scale
    assert float(np.abs(uh[0, 0, 0]).max()) <= 1e-15 * scale


def test_biot_savart_zeroes_mean_and_nyquist():
    N = 8
    w = fields.spectrum_modes(N, kc=3.0, seed=2, nyquist=True)
    uh = sp.velocity_modes(w, sp.VORTICITY)  # [a][k3][k2][k1]
    assert np.all(uh[:, 0, 0, 0] == 0)
    assert np.all(uh[:, N // 2] == 0) and np.all(uh[:, :, N // 2] == 0) and np.all(uh[:, :, :, N // 2] == 0)


def test_generator_structure():
    N = 12
    s = fields.spectrum_modes(N, kc=4.0, seed=5)
    r = (-np.arange(N)) % N
    for k1 in (0, N // 2):
        P = s[:, :, k1, :]
        assert np.array_equal(P, np.conj(P[r][:, r]))  # exactly Hermitian
    idx = np.arange(N)
    assert np.all(s[N // 2] == 0) and np.all(s[:, N // 2] == 0) and np.all(s[:, :, N // 2] == 0)
    kf = np.fft.fftfreq(N, d=1.0 / N)
    kdot = (np.arange(N // 2 + 1)[None, None, :] * s[..., 0] + kf[:, None, None] * s[..., 1]
            + kf[None, :, None] * s[..., 2])
    assert float(np.abs(kdot).max()) < 1e-12
    sn = fields.spectrum_modes(N, kc=4.0, seed=5, nyquist=True)
    assert np.any(sn[N // 2] != 0)
    P = sn[:, :, N // 2, :]
    assert np.array_equal(P, np.conj(P[r][:, r]))
    assert idx.size == N
