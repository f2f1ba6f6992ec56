"""Exact 1-D interpolation kernels beta_j(t) (oracle; test infrastructure only).

The paper writes the interpolant as a tensor-product sum over I nodes per axis,
i = 1-I/2 .. I/2, weighted by polynomials beta_i of the in-cell offset
t = xbar/delta (Sec. 2.2, Eq. "triple_sum").  It names two families: Lagrange
polynomials (Sec. 2.2, "for testing purposes", textbook Sec. 3.1 of the cited
numerical-analysis book) and local spline kernels of smoothness m (Sec. 2.2,
cited to the authors' earlier spline paper, whose tables are not reproduced in
the paper).

Readings taken here (the paper is silent on the spline construction):

* Nodes j = -n .. n+1 with I = 2n+2, t in [0, 1).  Only even I is defined,
  because the paper's index range is symmetric about the cell only for even I.
* Lagrange: beta_j(t) = prod_{k != j} (t-k)/(j-k).
* Spline (n, m), 0 <= m <= n: beta_j is the degree-(2n+1) polynomial p on
  [0, 1] fixed by
    - p(0) = f_0, p(1) = f_1;
    - for k = 1..m: p^(k)(0) is the k-th derivative at 0 of the degree-2n
      Lagrange interpolant through nodes -n..n, and p^(k)(1) the k-th derivative
      at 1 of the one through nodes 1-n..n+1 (a centred finite difference shared
      by both cells that meet at a node, which makes the piecewise interpolant
      exactly C^m);
    - p(r) = f_r at the 2(n-m) nodes nearest the cell,
      r in {-(n-m)..-1} U {2..n-m+1};
  evaluated with f = e_j.  m = 0 gives the Lagrange kernel; (n, m) = (1, 1) is
  the Catmull-Rom kernel.  Parity with the authors' published spline tables is
  unpinned (those tables are not available); the construction is pinned by its
  invariants in the tests.

All arithmetic is exact (``fractions.Fraction``).  Polynomials are lists of
coefficients in ascending powers of t.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from typing import List, Sequence, Tuple

Poly = List[Fraction]


def nodes(I: int) -> List[int]:
    """Node offsets j = 1-I/2 .. I/2 of an I-point kernel (Sec. 2.2)."""
    if I < 2 or I % 2:
        raise ValueError("only even kernel sizes I >= 2 are defined")
    n = I // 2 - 1
    return list(range(-n, n + 2))


def poly_mul(a: Sequence[Fraction], b: Sequence[Fraction]) -> Poly:
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def poly_eval(p: Sequence[Fraction], t) -> Fraction:
    """Exact value of p at t (t converted exactly to a Fraction)."""
    t = Fraction(t)
    acc = Fraction(0)
    for c in reversed(p):
        acc = acc * t + c
    return acc


def poly_deriv(p: Sequence[Fraction], k: int = 1) -> Poly:
    out = list(p)
    for _ in range(k):
        out = [i * out[i] for i in range(1, len(out))] or [Fraction(0)]
    return out


def lagrange_basis(node_list: Sequence[int], j: int) -> Poly:
    """Textbook Lagrange basis polynomial that is 1 at node j, 0 at the others."""
    p: Poly = [Fraction(1)]
    for k in node_list:
        if k == j:
            continue
        p = poly_mul(p, [Fraction(-k, j - k), Fraction(1, j - k)])
    return p


@lru_cache(maxsize=None)
def lagrange_kernel(I: int) -> Tuple[Tuple[Fraction, ...], ...]:
    """beta_j for the I-point Lagrange kernel, j in nodes(I)."""
    ns = nodes(I)
    return tuple(tuple(lagrange_basis(ns, j)) for j in ns)


def _solve(A: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    """Exact Gauss-Jordan elimination with row pivoting."""
    n = len(A)
    M = [list(row) + [rhs] for row, rhs in zip(A, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [v / pv for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[col])]
    return [M[r][n] for r in range(n)]


def _deriv_row(deg: int, k: int, x: int) -> List[Fraction]:
    """Row of the k-th derivative functional at x acting on monomial coefficients."""
    row = []
    for i in range(deg + 1):
        if i < k:
            row.append(Fraction(0))
            continue
        f = 1
        for r in range(k):
            f *= i - r
        row.append(Fraction(f) * Fraction(x) ** (i - k))
    return row


@lru_cache(maxsize=None)
def spline_kernel(I: int, m: int) -> Tuple[Tuple[Fraction, ...], ...]:
    """beta_j for the I-point, C^m spline kernel (construction in module doc)."""
    ns = nodes(I)
    n = I // 2 - 1
    if not 0 <= m <= n:
        raise ValueError("smoothness m must satisfy 0 <= m <= I/2 - 1")
    deg = 2 * n + 1
    left = list(range(-n, n + 1))        # stencil whose polynomial fixes p^(k)(0)
    right = list(range(1 - n, n + 2))    # stencil whose polynomial fixes p^(k)(1)
    extra = list(range(-(n - m), 0)) + list(range(2, n - m + 2))
    rows: List[List[Fraction]] = []
    rows.append(_deriv_row(deg, 0, 0))
    rows.append(_deriv_row(deg, 0, 1))
    for k in range(1, m + 1):
        rows.append(_deriv_row(deg, k, 0))
        rows.append(_deriv_row(deg, k, 1))
    for r in extra:
        rows.append(_deriv_row(deg, 0, r))
    assert len(rows) == deg + 1
    out = []
    for j in ns:
        rhs = [Fraction(int(j == 0)), Fraction(int(j == 1))]
        for k in range(1, m + 1):
            dl = poly_eval(poly_deriv(lagrange_basis(left, j), k), 0) if j in left else Fraction(0)
            dr = poly_eval(poly_deriv(lagrange_basis(right, j), k), 1) if j in right else Fraction(0)
            rhs += [dl, dr]
        for r in extra:
            rhs.append(Fraction(int(j == r)))
        out.append(tuple(_solve(rows, rhs)))
    return tuple(out)


LAGRANGE, SPLINE = 0, 1


def kernel(family: int, I: int, m: int = 0) -> Tuple[Tuple[Fraction, ...], ...]:
    """Exact beta_j polynomials for a kernel family (LAGRANGE or SPLINE)."""
    if family == LAGRANGE:
        return lagrange_kernel(I)
    if family == SPLINE:
        return spline_kernel(I, m)
    raise ValueError("unknown kernel family")


def derivative_kernel(family: int, I: int, m: int = 0) -> Tuple[Tuple[Fraction, ...], ...]:
    """d beta_j / dt, the derivative kernels used for velocity gradients."""
    return tuple(tuple(poly_deriv(list(p))) for p in kernel(family, I, m))


def weights_exact(family: int, I: int, m: int, t, deriv: bool = False) -> List[Fraction]:
    """Exact beta_j(t) (or beta_j'(t)) for all nodes, t taken exactly."""
    ker = derivative_kernel(family, I, m) if deriv else kernel(family, I, m)
    return [poly_eval(p, t) for p in ker]


def coeff_table_f64(family: int, I: int, m: int, deriv: bool = False):
    """Coefficient table [I][I] as float64 (each exact rational rounded once)."""
    import numpy as np
    ker = derivative_kernel(family, I, m) if deriv else kernel(family, I, m)
    tab = np.zeros((I, I), dtype=np.float64)
    for j, p in enumerate(ker):
        for i, c in enumerate(p):
            tab[j, i] = float(c)
    return tab
