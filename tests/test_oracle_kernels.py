"""Pins of the oracle's kernel polynomials (CPU only).

Each check is something the kernels must satisfy independently of how the
oracle builds them: textbook closed forms, golden check values, partition of
unity, polynomial reproduction, interpolation at the nodes, symmetry and exact
C^m continuity of the piecewise interpolant.
"""
import os
from fractions import Fraction as Fr

import pytest

from oracle import kernels as K

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kernel_values_t025.txt")
CASES = [(K.LAGRANGE, 4, 0), (K.LAGRANGE, 6, 0), (K.LAGRANGE, 8, 0),
         (K.SPLINE, 4, 1), (K.SPLINE, 6, 1), (K.SPLINE, 6, 2), (K.SPLINE, 8, 1),
         (K.SPLINE, 8, 2), (K.SPLINE, 8, 3)]


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, vals = line.split(":")
        fam, I, m, kind = head.split()
        rows.append((K.LAGRANGE if fam == "lagrange" else K.SPLINE, int(I), int(m),
                     kind, [Fr(v) for v in vals.split()]))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}-{r[3]}")
def test_golden_values_at_quarter(row):
    fam, I, m, kind, vals = row
    got = K.weights_exact(fam, I, m, Fr(1, 4), deriv=(kind == "deriv"))
    assert got == vals


def test_lagrange4_textbook_closed_form():
    # the four cubic Lagrange basis polynomials on nodes -1, 0, 1, 2, typed by hand
    forms = [lambda t: -t * (t - 1) * (t - 2) / 6,
             lambda t: (t + 1) * (t - 1) * (t - 2) / 2,
             lambda t: -(t + 1) * t * (t - 2) / 2,
             lambda t: (t + 1) * t * (t - 1) / 6]
    for t in [Fr(0), Fr(1, 3), Fr(5, 7), Fr(99, 100)]:
        assert K.weights_exact(K.LAGRANGE, 4, 0, t) == [f(t) for f in forms]


def test_catmull_rom_closed_form():
    forms = [lambda t: (-t ** 3 + 2 * t ** 2 - t) / 2,
             lambda t: (3 * t ** 3 - 5 * t ** 2 + 2) / 2,
             lambda t: (-3 * t ** 3 + 4 * t ** 2 + t) / 2,
             lambda t: (t ** 3 - t ** 2) / 2]
    for t in [Fr(0), Fr(1, 3), Fr(5, 7), Fr(99, 100)]:
        assert K.weights_exact(K.SPLINE, 4, 1, t) == [f(t) for f in forms]


@pytest.mark.parametrize("I", [4, 6, 8])
def test_spline_m0_is_lagrange(I):
    assert K.spline_kernel(I, 0) == K.lagrange_kernel(I)


@pytest.mark.parametrize("fam,I,m", CASES)
def test_partition_of_unity_and_degree(fam, I, m):
    ker = K.kernel(fam, I, m)
    assert all(len(p) <= I for p in ker)            # degree <= I-1
    total = [sum(p[i] for p in ker) for i in range(I)]
    assert total == [Fr(1)] + [Fr(0)] * (I - 1)


@pytest.mark.parametrize("fam,I,m", CASES)
def test_polynomial_reproduction(fam, I, m):
    # sum_j beta_j(t) j^r == t^r for r up to the reproduction degree:
    # I-1 for Lagrange, I-2 for the splines (m >= 1)
    top = I - 1 if (fam == K.LAGRANGE or m == 0) else I - 2
    js = K.nodes(I)
    for r in range(top + 1):
        for t in [Fr(1, 5), Fr(2, 3), Fr(7, 8)]:
            w = K.weights_exact(fam, I, m, t)
            assert sum(wj * Fr(j) ** r for wj, j in zip(w, js)) == t ** r
    if fam == K.SPLINE and m >= 1:
        # and not one degree more (the splines trade one order for smoothness)
        t = Fr(1, 5)
        w = K.weights_exact(fam, I, m, t)
        assert sum(wj * Fr(j) ** (top + 1) for wj, j in zip(w, js)) != t ** (top + 1)


@pytest.mark.parametrize("fam,I,m", CASES)
def test_interpolates_at_cell_ends(fam, I, m):
    js = K.nodes(I)
    assert K.weights_exact(fam, I, m, 0) == [Fr(int(j == 0)) for j in js]
    assert K.weights_exact(fam, I, m, 1) == [Fr(int(j == 1)) for j in js]


@pytest.mark.parametrize("fam,I,m", CASES)
def test_mirror_symmetry(fam, I, m):
    js = K.nodes(I)
    for t in [Fr(1, 7), Fr(3, 10)]:
        w = dict(zip(js, K.weights_exact(fam, I, m, t)))
        wm = dict(zip(js, K.weights_exact(fam, I, m, 1 - t)))
        assert all(w[j] == wm[1 - j] for j in js)


@pytest.mark.parametrize("fam,I,m", CASES)
def test_exact_cm_continuity(fam, I, m):
    """Derivatives 0..m of the piecewise interpolant agree across a node.

    On cell [0,1] datum f_j carries weight beta_j(t); on cell [1,2] the same
    datum carries beta_{j-1}(t-1).  Continuity at x = 1 of the k-th derivative
    for arbitrary data means beta_j^(k)(1) == beta_{j-1}^(k)(0) for every j
    (a weight outside a stencil is zero).
    """
    ker = dict(zip(K.nodes(I), K.kernel(fam, I, m)))
    order = m if (fam == K.SPLINE) else 0

    def d(j, k, x):
        return K.poly_eval(K.poly_deriv(list(ker[j]), k), x) if j in ker else Fr(0)

    js = list(range(min(ker) - 1, max(ker) + 2))
    for k in range(order + 1):
        assert all(d(j, k, 1) == d(j - 1, k, 0) for j in js), k
    # the next derivative jumps (so the stated smoothness is the true one)
    assert any(d(j, order + 1, 1) != d(j - 1, order + 1, 0) for j in js)


@pytest.mark.parametrize("fam,I,m", CASES)
def test_derivative_kernel_moments(fam, I, m):
    js = K.nodes(I)
    for t in [Fr(1, 9), Fr(1, 2), Fr(4, 5)]:
        dw = K.weights_exact(fam, I, m, t, deriv=True)
        assert sum(dw) == 0
        assert sum(w * j for w, j in zip(dw, js)) == 1


def test_odd_sizes_rejected():
    with pytest.raises(ValueError):
        K.nodes(5)
    with pytest.raises(ValueError):
        K.spline_kernel(6, 3)


# ---- the spline reading rebuilt by a second, independent construction: Hermite
# interpolation in Newton form (confluent divided differences) of the data
# e_j, with the end derivatives taken from centred Lagrange interpolants built
# by ordinary divided differences.  The oracle solves a linear system in the
# monomial basis instead; the two share no code.

def _newton(xs, ys):
    """Divided-difference coefficients on distinct nodes xs."""
    c = list(ys)
    for k in range(1, len(xs)):
        for i in range(len(xs) - 1, k - 1, -1):
            c[i] = (c[i] - c[i - 1]) / (xs[i] - xs[i - k])
    return c


def _newton_deriv_at(xs, c, x, k):
    """k-th derivative at x of sum_i c_i prod_{l<i} (t - xs_l), by expanding the
    products into ascending coefficients."""
    poly = [Fr(0)] * len(c)
    basis = [Fr(1)]
    for i, ci in enumerate(c):
        for p, b in enumerate(basis):
            poly[p] += ci * b
        nxt = [Fr(0)] * (len(basis) + 1)
        for p, b in enumerate(basis):
            nxt[p + 1] += b
            nxt[p] -= xs[i] * b
        basis = nxt
    tot = Fr(0)
    for p in range(k, len(poly)):
        fall = 1
        for q in range(k):
            fall *= p - q
        tot += poly[p] * fall * Fr(x) ** (p - k)
    return tot


def _hermite_eval(zs, derivs, t):
    """Hermite interpolant in Newton form: zs sorted with repeats, derivs[z][k]
    the k-th derivative at node z; evaluated at t."""
    n = len(zs)
    table = [[Fr(0)] * n for _ in range(n)]
    for i in range(n):
        table[i][0] = derivs[zs[i]][0]
    for k in range(1, n):
        for i in range(n - k):
            if zs[i + k] == zs[i]:
                f = 1
                for q in range(2, k + 1):
                    f *= q
                table[i][k] = derivs[zs[i]][k] / f
            else:
                table[i][k] = (table[i + 1][k - 1] - table[i][k - 1]) / (zs[i + k] - zs[i])
    val, prod = Fr(0), Fr(1)
    for k in range(n):
        val += table[0][k] * prod
        prod *= (t - zs[k])
    return val


def _spline_weight_hermite(I, m, j, t):
    n = I // 2 - 1
    data = {x: Fr(int(x == j)) for x in range(-n - 1, n + 3)}
    left = list(range(-n, n + 1))
    right = list(range(1 - n, n + 2))
    cl = _newton(left, [data[x] for x in left])
    cr = _newton(right, [data[x] for x in right])
    derivs = {0: [data[0]] + [_newton_deriv_at(left, cl, 0, k) for k in range(1, m + 1)],
              1: [data[1]] + [_newton_deriv_at(right, cr, 1, k) for k in range(1, m + 1)]}
    extra = list(range(-(n - m), 0)) + list(range(2, n - m + 2))
    for r in extra:
        derivs[r] = [data[r]]
    zs = sorted(extra + [0] * (m + 1) + [1] * (m + 1))
    return _hermite_eval(zs, derivs, Fr(t))


@pytest.mark.parametrize("I,m", [(4, 1), (6, 1), (6, 2), (8, 1), (8, 2), (8, 3)])
def test_spline_matches_hermite_newton_construction(I, m):
    for t in [Fr(1, 4), Fr(2, 3), Fr(9, 10)]:
        got = K.weights_exact(K.SPLINE, I, m, t)
        want = [_spline_weight_hermite(I, m, j, t) for j in K.nodes(I)]
        assert got == want
