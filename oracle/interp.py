"""Step 4 of the interpolation algorithm: the weighted triple sum (oracle).

Test infrastructure only.  Follows Sec. 2.2, Eq. "triple_sum":

    u(X) ~= sum_{i1,i2,i3 = 1-I/2}^{I/2} beta_i1(t1) beta_i2(t2) beta_i3(t3) u(c + i)

with indices taken modulo N (periodic domain), and the velocity gradient read as
the same sum with beta replaced by its derivative on the differentiated axis,
times d t/d x = 1/delta (= invd, the constant of ``geometry``).

Field layout: ``u[x3][x2][x1][a]`` (x1 fastest, component fastest within a
node), a numpy array of shape (N, N, N, 3).  Positions ``X[p] = (x1, x2, x3)``.
Gradient layout: ``grad[p][a][b] = d u_a / d x_b``.

Two independent evaluations are provided: ``interp_brute`` (explicit loops,
exact-rational weights rounded once) for tiny cases and ``interp_vec``
(vectorised gather + einsum, weights by FP64 Horner) for the rest.  All sums are
FP64.
"""
from __future__ import annotations

import numpy as np

from . import geometry, kernels


def weights_f64(family: int, I: int, m: int, t: np.ndarray, deriv: bool = False) -> np.ndarray:
    """beta_j(t) for every entry of t by Horner in FP64, shape t.shape + (I,)."""
    tab = kernels.coeff_table_f64(family, I, m, deriv)  # [j][power]
    t = np.asarray(t, dtype=np.float64)
    out = np.empty(t.shape + (I,), dtype=np.float64)
    for j in range(I):
        acc = np.full(t.shape, tab[j, I - 1])
        for p in range(I - 2, -1, -1):
            acc = np.add(np.multiply(acc, t), tab[j, p])
        out[..., j] = acc
    return out


def weights_abs(family: int, I: int, m: int, t: np.ndarray, deriv: bool = False) -> np.ndarray:
    """H_j(t) = sum_p |c_jp| t^p (t >= 0) for the coefficients c_jp of beta_j
    (or beta_j'): it bounds |beta_j(t)| and, times the number of Horner steps
    and the unit roundoff, the rounding error of any Horner evaluation of
    beta_j(t) (the standard bound for Horner's rule), so sums of |terms| built
    from it bound reduced-precision evaluations of the kernel."""
    tab = np.abs(kernels.coeff_table_f64(family, I, m, deriv))
    t = np.asarray(t, dtype=np.float64)
    out = np.empty(t.shape + (I,), dtype=np.float64)
    for j in range(I):
        acc = np.full(t.shape, tab[j, I - 1])
        for p in range(I - 2, -1, -1):
            acc = np.add(np.multiply(acc, np.abs(t)), tab[j, p])
        out[..., j] = acc
    return out


def _gather(field: np.ndarray, c: np.ndarray, I: int) -> np.ndarray:
    """Stencil values [P, I(x3), I(x2), I(x1), 3] around cells c[P, 3]."""
    N = field.shape[0]
    off = np.arange(1 - I // 2, I // 2 + 1)
    i1 = (c[:, 0, None] + off) % N
    i2 = (c[:, 1, None] + off) % N
    i3 = (c[:, 2, None] + off) % N
    return field[i3[:, :, None, None], i2[:, None, :, None], i1[:, None, None, :]]


def interp_vec(field: np.ndarray, X: np.ndarray, family: int, I: int, m: int = 0,
               gradient: bool = False, chunk: int = 4096, absolute: bool = False):
    """Vectorised triple sum; returns u[P,3] (and grad[P,3,3] if requested).

    With ``absolute=True`` every field value is replaced by its absolute value
    and every weight by ``weights_abs`` (the sum of the absolute values of its
    polynomial's terms): the result bounds the size of every term and partial
    sum and of the Horner rounding of the weights, for any evaluation order
    (used to derive tolerances for reduced-precision arithmetic).
    """
    field = np.asarray(field)           # FP32 or FP64 values; gathered stencils become FP64
    if absolute:
        field = np.abs(field)
    N = field.shape[0]
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    P = X.shape[0]
    u = np.empty((P, 3))
    g = np.empty((P, 3, 3)) if gradient else None
    invd = geometry.inv_delta(N)
    for s in range(0, P, chunk):
        e = min(P, s + chunk)
        c, t = geometry.cell_and_offset(X[s:e], N)
        w = weights_abs(family, I, m, t) if absolute else weights_f64(family, I, m, t)  # [p, axis, I]
        G = _gather(field, c, I).astype(np.float64)  # [p, k3, k2, k1, a]
        u[s:e] = np.einsum("pk,pj,pi,pkjia->pa", w[:, 2], w[:, 1], w[:, 0], G)
        if gradient:
            d = (weights_abs(family, I, m, t, deriv=True) if absolute
                 else weights_f64(family, I, m, t, deriv=True)) * invd
            g[s:e, :, 0] = np.einsum("pk,pj,pi,pkjia->pa", w[:, 2], w[:, 1], d[:, 0], G)
            g[s:e, :, 1] = np.einsum("pk,pj,pi,pkjia->pa", w[:, 2], d[:, 1], w[:, 0], G)
            g[s:e, :, 2] = np.einsum("pk,pj,pi,pkjia->pa", d[:, 2], w[:, 1], w[:, 0], G)
    return (u, g) if gradient else u


def interp_brute(field, X, family: int, I: int, m: int = 0, gradient: bool = False):
    """Explicit-loop triple sum, weights exact rationals rounded once to FP64."""
    field = np.asarray(field, dtype=np.float64)
    N = field.shape[0]
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    invd = geometry.inv_delta(N)
    offs = kernels.nodes(I)
    us, gs = [], []
    for p in range(X.shape[0]):
        cs, ts = [], []
        for d in range(3):
            c, t = geometry.cell_and_offset_scalar(float(X[p, d]), N)
            cs.append(c)
            ts.append(t)
        w = [[float(v) for v in kernels.weights_exact(family, I, m, ts[d])] for d in range(3)]
        dw = [[float(v) * invd for v in kernels.weights_exact(family, I, m, ts[d], True)]
              for d in range(3)] if gradient else None
        acc = [0.0, 0.0, 0.0]
        gacc = [[0.0] * 3 for _ in range(3)]
        for k3, i3 in enumerate(offs):
            for k2, i2 in enumerate(offs):
                for k1, i1 in enumerate(offs):
                    node = field[(cs[2] + i3) % N, (cs[1] + i2) % N, (cs[0] + i1) % N]
                    wv = w[0][k1] * w[1][k2] * w[2][k3]
                    for a in range(3):
                        acc[a] += wv * node[a]
                    if gradient:
                        gw = (dw[0][k1] * w[1][k2] * w[2][k3],
                              w[0][k1] * dw[1][k2] * w[2][k3],
                              w[0][k1] * w[1][k2] * dw[2][k3])
                        for a in range(3):
                            for b in range(3):
                                gacc[a][b] += gw[b] * node[a]
        us.append(acc)
        gs.append(gacc)
    u = np.array(us, dtype=np.float64).reshape(-1, 3)
    if gradient:
        return u, np.array(gs, dtype=np.float64).reshape(-1, 3, 3)
    return u
