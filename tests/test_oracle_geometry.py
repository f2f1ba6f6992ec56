"""Pins of the oracle's wrap / cell / bin / order / offsets (CPU only)."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import geometry as G

L = G.L


def _tol(x: float, N: int) -> float:
    """Rounding bound on t: a few ulps of max(|x|, L), scaled to cell units."""
    return 4 * 2.0 ** -52 * max(abs(x), L) * N / L + 2.0 ** -50


def _exact_cell(x: float, N: int):
    """Cell and offset in exact rational arithmetic with L = fl64(2*pi) exactly."""
    Lr = Fr(L)
    xr = Fr(x)
    y = xr - Lr * math.floor(xr / Lr)
    s = y * N / Lr
    c = math.floor(s)
    return c % N, s - c


EDGE = [0.0, -0.0, -1e-300, 5e-324, L, math.nextafter(L, 0.0), math.nextafter(L, 10.0),
        -L, 3 * L, math.nextafter(3 * L, 0.0), math.nextafter(-2 * L, 0.0), 1e6, -1e6,
        12345.678, -0.5, 1.0, math.pi, math.nextafter(0.0, -1.0)]


@pytest.mark.parametrize("N", [8, 9, 32, 1024])
def test_edge_cases_valid_and_match_exact(N):
    for x in EDGE:
        c, t = G.cell_and_offset_scalar(x, N)
        assert 0 <= c < N and 0.0 <= t < 1.0, (x, c, t)
        ce, te = _exact_cell(x, N)
        # the binary64 sequence may only differ from exact arithmetic by landing
        # on the neighbouring cell when the exact point is within rounding of a face
        if ce != c:
            assert (ce - c) % N in (1, N - 1), (x, c, ce)
            assert min(te, 1 - te) < _tol(x, N) or min(t, 1 - t) < _tol(x, N), (x, t, te)
        else:
            assert abs(float(te) - t) < _tol(x, N), (x, t, te)


def test_specific_edge_values():
    N = 32
    assert G.cell_and_offset_scalar(-1e-300, N) == (0, 0.0)   # -tiny + L rounds to L -> 0
    assert G.cell_and_offset_scalar(L, N) == (0, 0.0)
    assert G.cell_and_offset_scalar(-0.0, N) == (0, 0.0)
    c, t = G.cell_and_offset_scalar(math.nextafter(L, 0.0), N)
    assert (c, t) in ((0, 0.0),) or (c == N - 1 and t > 0.999999)


def test_node_positions_give_zero_offset():
    for N in [8, 12, 32, 256, 1024]:
        invd = G.inv_delta(N)
        for j in [0, 1, N // 3, N - 1]:
            x = j / invd
            c, t = G.cell_and_offset_scalar(x, N)
            # x = j/invd need not round-trip; when it does, t is exactly 0
            if x * invd == float(j):
                assert (c, t) == (j, 0.0)


def test_vector_matches_scalar():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(-50, 50, 5000), np.array(EDGE)])
    for N in [9, 64]:
        c, t = G.cell_and_offset(x, N)
        for i in range(len(x)):
            assert (int(c[i]), float(t[i])) == G.cell_and_offset_scalar(float(x[i]), N)


def test_random_points_match_exact_rational():
    rng = np.random.default_rng(7)
    x = rng.uniform(-20, 20, 3000)
    for N in [16, 1024]:
        c, t = G.cell_and_offset(x, N)
        for i in range(len(x)):
            ce, te = _exact_cell(float(x[i]), N)
            if ce == c[i]:
                assert abs(float(te) - t[i]) < _tol(float(x[i]), N)
            else:
                assert min(float(te), 1 - float(te)) < _tol(float(x[i]), N)


def test_wrap_range():
    x = np.array(EDGE + [1e15, -1e15])
    y = G.wrap(x)
    assert np.all((y >= 0) & (y < L))


def test_keys_order_offsets_against_naive():
    rng = np.random.default_rng(11)
    for N, T, W, Np in [(8, 8, 4, 50), (9, 16, 4, 200), (32, 16, 4, 3000), (24, 8, 4, 1000), (40, 16, 4, 700)]:
        X = rng.uniform(-L, 2 * L, (Np, 3))
        keys = G.bin_keys(X, N, T, W)
        ntx, nw = -(-N // T), -(-N // W)
        nbins = G.n_bins(N, T, W)
        assert nbins == ntx * ntx * nw
        # naive key from per-axis scalar cells: column (x2 tile, x1 tile), then x3 window
        for p in range(0, Np, 37):
            cs = [G.cell_and_offset_scalar(float(X[p, d]), N)[0] for d in range(3)]
            column = (cs[1] // T) * ntx + cs[0] // T
            assert keys[p] == column * nw + cs[2] // W
            assert 0 <= keys[p] < nbins
        perm = G.stable_order(keys)
        assert list(perm) == G.naive_stable_order(keys)
        off = G.offsets_from_keys(keys, nbins)
        assert off[0] == 0 and off[-1] == Np and len(off) == nbins + 1
        for b in range(nbins):
            assert off[b + 1] - off[b] == sum(1 for k in keys if k == b)
