"""Pins of the oracle's triple sum and gradient (CPU only).

The oracle's two evaluations (explicit loops with exact weights, vectorised
gather with Horner weights) and the plain-C version are compared with each
other, and all of them with results the mathematics fixes: constants, nodes,
polynomial reproduction, separable products, the closed-form transfer function
of a single Fourier mode, convergence orders, and finite differences.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import cbuild, geometry, interp
from oracle import kernels as K
from synthetic import fields

L = geometry.L
KERNELS = [(K.LAGRANGE, 4, 0), (K.SPLINE, 6, 1), (K.SPLINE, 8, 2), (K.LAGRANGE, 8, 0)]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.sqrt(np.mean(b * b)), 1e-300))


@pytest.mark.parametrize("N", [8, 9, 12])
@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_brute_vec_c_agree(N, fam, I, m):
    rng = np.random.default_rng(N * 100 + I)
    u = rng.standard_normal((N, N, N, 3))
    X = rng.uniform(-L, 2 * L, (12, 3))
    ub, gb = interp.interp_brute(u, X, fam, I, m, gradient=True)
    uv, gv = interp.interp_vec(u, X, fam, I, m, gradient=True)
    uc, gc, _ = cbuild.triple_sum(u, X, fam, I, m, gradient=True)
    assert _rel(uv, ub) < 1e-13 and _rel(gv, gb) < 1e-13
    assert _rel(uc, ub) < 1e-13 and _rel(gc, gb) < 1e-13


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_constant_field(fam, I, m):
    N = 16
    u = np.empty((N, N, N, 3))
    u[...] = [1.5, -2.25, 0.125]
    X = np.random.default_rng(1).uniform(0, L, (200, 3))
    val, grad = interp.interp_vec(u, X, fam, I, m, gradient=True)
    assert np.max(np.abs(val - u[0, 0, 0])) < 1e-14
    assert np.max(np.abs(grad)) < 1e-11


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_node_values_exact(fam, I, m):
    N = 12
    rng = np.random.default_rng(2)
    u = rng.standard_normal((N, N, N, 3))
    invd = geometry.inv_delta(N)
    idx = rng.integers(0, N, (50, 3))
    X = idx / invd
    ok = np.all(X * invd == idx, axis=1)          # positions whose t is exactly 0
    val = interp.interp_vec(u, X[ok], fam, I, m)
    ref = u[idx[ok, 2], idx[ok, 1], idx[ok, 0]]
    assert ok.sum() > 10
    assert np.array_equal(val, ref)


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_polynomial_reproduction_3d(fam, I, m):
    # f(node) = polynomial of the node's integer coordinates, of degree up to the
    # kernel's reproduction degree per axis; particles away from the periodic seam
    deg = I - 1 if fam == K.LAGRANGE else I - 2
    N = 32
    g = np.arange(N, dtype=np.float64)
    Z, Y, Xg = np.meshgrid(g, g, g, indexing="ij")
    cx = [0.5, -0.25, 0.75]

    def poly(x, y, z, a):
        return cx[a] * (x / 8) ** deg + (y / 8) ** (deg - 1) * (z / 8) + a * (z / 8) ** deg - 0.3

    u = np.stack([poly(Xg, Y, Z, a) for a in range(3)], axis=-1)
    rng = np.random.default_rng(3)
    sgrid = rng.uniform(I, N - I, (100, 3))          # in grid units, no wrap
    X = sgrid / geometry.inv_delta(N)
    c, t = geometry.cell_and_offset(X, N)
    s = c + t
    exact = np.stack([poly(s[:, 0], s[:, 1], s[:, 2], a) for a in range(3)], axis=-1)
    val = interp.interp_vec(u, X, fam, I, m)
    assert np.max(np.abs(val - exact)) < 1e-9


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_separable_product_field(fam, I, m):
    N = 10
    rng = np.random.default_rng(4)
    f = [rng.standard_normal(N) for _ in range(3)]
    u = np.einsum("k,j,i->kji", f[2], f[1], f[0])[..., None] * np.array([1.0, -2.0, 0.5])
    X = rng.uniform(0, L, (40, 3))
    val = interp.interp_vec(u, X, fam, I, m)
    for p in range(X.shape[0]):
        prod = 1.0
        for d in range(3):
            c, t = geometry.cell_and_offset_scalar(float(X[p, d]), N)
            w = K.weights_exact(fam, I, m, Fr(t))
            prod *= float(sum(wj * Fr(float(f[d][(c + j) % N]))
                              for wj, j in zip(w, K.nodes(I))))
        assert np.allclose(val[p], prod * np.array([1.0, -2.0, 0.5]), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_single_mode_transfer_function(fam, I, m):
    """u = cos(k.x + phi): interpolant = Re(e^{i phi} prod_d sum_j beta_j e^{i k_d (c_d+j) delta})."""
    N = 16
    kvec = (2, -1, 3)
    u, _ = fields.single_mode_field(N, kvec, amp=(1.0, 1.0, 1.0), phase=(0.3, 0.3, 0.3))
    X = np.random.default_rng(6).uniform(0, L, (60, 3))
    val = interp.interp_vec(u, X, fam, I, m)
    delta = L / N
    for p in range(X.shape[0]):
        z = np.exp(0.3j)
        for d in range(3):
            c, t = geometry.cell_and_offset_scalar(float(X[p, d]), N)
            w = [float(v) for v in K.weights_exact(fam, I, m, Fr(t))]
            z *= sum(wj * np.exp(1j * kvec[d] * (c + j) * delta) for wj, j in zip(w, K.nodes(I)))
        assert abs(val[p, 0] - z.real) < 1e-12


@pytest.mark.parametrize("fam,I,m,order", [(K.LAGRANGE, 4, 0, 4), (K.SPLINE, 6, 1, 5),
                                           (K.SPLINE, 8, 2, 7), (K.LAGRANGE, 8, 0, 8)])
def test_convergence_order(fam, I, m, order):
    kvec = (1, 2, 1)
    X = np.random.default_rng(8).uniform(0, L, (400, 3))
    Ns = [16, 24, 32, 48]
    ev, eg = [], []
    for N in Ns:
        u, exact = fields.single_mode_field(N, kvec)
        val, grad = interp.interp_vec(u, X, fam, I, m, gradient=True)
        ex, gx = exact(X, gradient=True)
        ev.append(np.sqrt(np.mean((val - ex) ** 2)))
        eg.append(np.sqrt(np.mean((grad - gx) ** 2)))
    sv = -np.polyfit(np.log(Ns), np.log(ev), 1)[0]
    sg = -np.polyfit(np.log(Ns), np.log(eg), 1)[0]
    assert abs(sv - order) < 0.6, (sv, ev)
    assert abs(sg - (order - 1)) < 0.6, (sg, eg)


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_gradient_vs_central_difference(fam, I, m):
    N = 12
    rng = np.random.default_rng(9)
    u = rng.standard_normal((N, N, N, 3))
    invd = geometry.inv_delta(N)
    # points strictly inside cells so that x +- h stays in the same cell
    s = rng.integers(0, N, (20, 3)) + rng.uniform(0.2, 0.8, (20, 3))
    X = s / invd
    _, grad = interp.interp_vec(u, X, fam, I, m, gradient=True)
    h = 1e-5
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        fd = (interp.interp_vec(u, X + e, fam, I, m) - interp.interp_vec(u, X - e, fam, I, m)) / (2 * h)
        assert np.max(np.abs(fd - grad[:, :, b])) < 1e-6 * np.max(np.abs(grad))


def test_fourier_field_interpolation_error_drops():
    X = np.random.default_rng(10).uniform(0, L, (300, 3))
    errs = []
    for N in [32, 64]:
        u, modes = fields.fourier_mode_field(N, kmax=4, seed=0)
        ex = fields.fourier_mode_eval(modes, X)
        val = interp.interp_vec(u, X, K.SPLINE, 8, 2)
        errs.append(np.sqrt(np.mean((val - ex) ** 2)) / np.sqrt(np.mean(ex ** 2)))
    assert errs[1] < errs[0] / 30 and errs[1] < 1e-5


@pytest.mark.parametrize("fam,I,m", [(K.LAGRANGE, 4, 0), (K.SPLINE, 6, 1), (K.SPLINE, 8, 2)])
def test_absolute_weights_bound_the_weights(fam, I, m):
    """weights_abs (sum of |terms| of each kernel polynomial) is >= |beta|
    everywhere, equals |c_0| at t = 0, and the absolute interpolation sum
    bounds the value itself."""
    t = np.linspace(0.0, 0.999, 101)
    for deriv in (False, True):
        w = interp.weights_f64(fam, I, m, t, deriv)
        h = interp.weights_abs(fam, I, m, t, deriv)
        assert np.all(h >= np.abs(w) - 1e-15)
        c0 = np.abs(K.coeff_table_f64(fam, I, m, deriv)[:, 0])
        assert np.array_equal(h[0], c0)
    u = np.random.default_rng(1).standard_normal((12, 12, 12, 3))
    X = np.random.default_rng(2).uniform(0, 2 * np.pi, (300, 3))
    v, g = interp.interp_vec(u, X, fam, I, m, gradient=True)
    av, ag = interp.interp_vec(u, X, fam, I, m, gradient=True, absolute=True)
    assert np.all(av >= np.abs(v)) and np.all(ag >= np.abs(g))
