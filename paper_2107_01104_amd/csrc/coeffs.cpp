// Kernel-coefficient generator: the polynomials beta_j(t) of the I-point
// interpolation kernels (Sec. 2.2, Eq. "triple_sum": weights are polynomials of
// the in-cell offset t = xbar/delta) and their derivatives, derived here in
// exact rational arithmetic and rounded once to binary64 / binary32.
//
// Families (nodes j = -n..n+1, I = 2n+2):
//  * Lagrange: beta_j(t) = prod_{k != j} (t - k) / (j - k).
//  * Spline (n, m): on [0,1] the degree-(2n+1) polynomial p with
//      p(0) = f_0, p(1) = f_1,
//      p^(k)(0) = k-th derivative at 0 of the degree-2n Lagrange interpolant on
//                 nodes -n..n, p^(k)(1) likewise on nodes 1-n..n+1 (k = 1..m),
//      p(r) = f_r for r in {-(n-m)..-1} U {2..n-m+1},
//    applied to f = e_j.  m = 0 reproduces the Lagrange kernel.
//
// The conditions form a (2n+2)x(2n+2) linear system on the monomial
// coefficients of p; it is solved for all I right-hand sides at once by
// fraction-exact Gauss-Jordan elimination over __int128 rationals.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "ptk_internal.h"

namespace ptk {
namespace {

typedef __int128 i128;

i128 iabs(i128 a) { return a < 0 ? -a : a; }

i128 igcd(i128 a, i128 b) {
  a = iabs(a);
  b = iabs(b);
  while (b) {
    i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Rational number num/den with den > 0, always reduced.  Overflow of the
// __int128 intermediates sets a sticky flag instead of wrapping silently.
struct Q {
  i128 num = 0, den = 1;
};

bool g_overflow = false;

i128 mul_chk(i128 a, i128 b) {
  i128 r;
  if (__builtin_mul_overflow(a, b, &r)) g_overflow = true;
  return r;
}

i128 add_chk(i128 a, i128 b) {
  i128 r;
  if (__builtin_add_overflow(a, b, &r)) g_overflow = true;
  return r;
}

Q make(i128 n, i128 d = 1) {
  Q q;
  if (d < 0) {
    n = -n;
    d = -d;
  }
  i128 g = igcd(n, d);
  if (g > 1) {
    n /= g;
    d /= g;
  }
  q.num = n;
  q.den = d;
  return q;
}

Q operator+(Q a, Q b) {
  i128 g = igcd(a.den, b.den);
  i128 bd = b.den / g;
  return make(add_chk(mul_chk(a.num, bd), mul_chk(b.num, a.den / g)), mul_chk(a.den, bd));
}
Q operator-(Q a) { return make(-a.num, a.den); }
Q operator-(Q a, Q b) { return a + (-b); }
Q operator*(Q a, Q b) {
  i128 g1 = igcd(a.num, b.den), g2 = igcd(b.num, a.den);
  if (g1 == 0) g1 = 1;
  if (g2 == 0) g2 = 1;
  return make(mul_chk(a.num / g1, b.num / g2), mul_chk(a.den / g2, b.den / g1));
}
Q operator/(Q a, Q b) { return a * make(b.den, b.num); }
bool is_zero(Q a) { return a.num == 0; }

typedef std::vector<Q> Poly;  // ascending powers

// Coefficients of the Lagrange basis polynomial through `nodes` that is 1 at
// node `j`: expanded product of (t - k)/(j - k).
Poly lagrange_basis(const std::vector<int>& nodes, int j) {
  Poly p(1, make(1));
  for (int k : nodes) {
    if (k == j) continue;
    Poly q(p.size() + 1, make(0));
    Q inv = make(1, j - k);
    for (size_t i = 0; i < p.size(); ++i) {
      q[i + 1] = q[i + 1] + p[i] * inv;            // t * p
      q[i] = q[i] + p[i] * make(-k) * inv;          // -k * p
    }
    p = q;
  }
  return p;
}

// k-th derivative of p evaluated at integer x.
Q deriv_at(const Poly& p, int k, int x) {
  Q acc = make(0);
  for (int i = (int)p.size() - 1; i >= k; --i) {
    i128 f = 1;
    for (int r = 0; r < k; ++r) f *= (i - r);
    acc = acc * make(x) + p[i] * make(f);
  }
  return acc;
}

// Row of the functional "k-th derivative at x" on monomial coefficients
// 0..deg.
std::vector<Q> functional_row(int deg, int k, int x) {
  std::vector<Q> row(deg + 1, make(0));
  for (int i = k; i <= deg; ++i) {
    i128 f = 1;
    for (int r = 0; r < k; ++r) f *= (i - r);
    i128 xp = 1;
    for (int r = 0; r < i - k; ++r) xp *= x;
    row[i] = make(f * xp);
  }
  return row;
}

// Solve A X = B (A: n x n, B: n x n, row-major) exactly; returns false if
// singular or on overflow.
bool solve(std::vector<std::vector<Q>>& A, std::vector<std::vector<Q>>& B) {
  const int n = (int)A.size();
  for (int col = 0; col < n; ++col) {
    int piv = -1;
    for (int r = col; r < n; ++r)
      if (!is_zero(A[r][col])) {
        piv = r;
        break;
      }
    if (piv < 0) return false;
    std::swap(A[col], A[piv]);
    std::swap(B[col], B[piv]);
    Q inv = make(1) / A[col][col];
    for (int c = 0; c < n; ++c) A[col][c] = A[col][c] * inv;
    for (int c = 0; c < (int)B[col].size(); ++c) B[col][c] = B[col][c] * inv;
    for (int r = 0; r < n; ++r) {
      if (r == col || is_zero(A[r][col])) continue;
      Q f = A[r][col];
      for (int c = 0; c < n; ++c) A[r][c] = A[r][c] - f * A[col][c];
      for (int c = 0; c < (int)B[r].size(); ++c) B[r][c] = B[r][c] - f * B[col][c];
    }
  }
  return !g_overflow;
}

// Correctly rounded (to nearest, ties to even) conversion of an exact
// rational to a binary floating-point number with `bits` significand bits:
// the quotient is scaled by a power of two into [2^(bits-1), 2^bits) and
// rounded in integer arithmetic from its remainder.  The magnitudes of kernel
// coefficients keep every intermediate far inside __int128 and the result
// far inside the normal range.
bool to_binary(Q q, int bits, double* out) {
  if (q.num == 0) {
    *out = 0.0;
    return true;
  }
  const bool neg = q.num < 0;
  const i128 a = iabs(q.num), d = q.den;
  const int top = 124;  // keep a * 2^k and d * 2^k below 2^125
  int nb = 0, db = 0;
  for (i128 t = a; t; t >>= 1) ++nb;
  for (i128 t = d; t; t >>= 1) ++db;
  // e: the quotient a/d lies in [2^(nb-db-1), 2^(nb-db+1)); scale by 2^(-e)
  // so that it lies in [2^(bits-1), 2^(bits+1))
  int e = nb - db - bits;
  i128 num = a, den = d;
  if (e < 0) {
    if (nb - e > top) return false;
    num <<= -e;
  } else {
    if (db + e > top) return false;
    den <<= e;
  }
  i128 quo = num / den, rem = num % den;
  if (quo >= ((i128)1 << bits)) {  // one bit too many: halve, folding the dropped bit into the remainder
    const i128 lowbit = quo & 1;
    quo >>= 1;
    rem = lowbit * den + rem;
    den <<= 1;
    ++e;
  }
  const i128 twice = 2 * rem;
  if (twice > den || (twice == den && (quo & 1))) ++quo;  // a carry to 2^bits stays exact
  double v = (double)(int64_t)quo;
  v = ldexp(v, e);
  *out = neg ? -v : v;
  return true;
}

bool to_double(Q q, double* out) { return to_binary(q, 53, out); }

bool to_float(Q q, float* out) {
  double v;
  if (!to_binary(q, 24, &v)) return false;
  *out = (float)v;  // exact: v already has at most 24 significand bits
  return true;
}

// The same polynomial in powers of (t - 1/2): coefficient q is
// sum_{p >= q} c_p C(p, q) (1/2)^(p - q).
Poly centred(const Poly& c) {
  const int n = (int)c.size();
  Poly d(n, make(0));
  for (int q = 0; q < n; ++q)
    for (int p = q; p < n; ++p) {
      i128 binom = 1;
      for (int r = 0; r < q; ++r) binom = binom * (p - r) / (r + 1);
      d[q] = d[q] + c[p] * make(binom, (i128)1 << (p - q));
    }
  return d;
}

}  // namespace

// Fill the coefficient tables of a kernel: val[j][p] and der[j][p] (node j in
// 0..I-1 standing for offset j - (I/2-1), power p ascending).  Returns 0, or
// PTK_EUNSUPPORTED / PTK_EINVAL.
int build_kernel_tables(int family, int I, int m, KernelTables* out) {
  if (I < 2 || I % 2 != 0 || I > kMaxI) return -6;
  const int n = I / 2 - 1;
  if (family == 0) m = 0;
  if (family != 0 && family != 1) return -1;
  if (m < 0 || m > n) return -1;
  g_overflow = false;
  const int deg = 2 * n + 1;
  std::vector<int> all, left, right;
  for (int j = -n; j <= n + 1; ++j) all.push_back(j);
  for (int j = -n; j <= n; ++j) left.push_back(j);
  for (int j = 1 - n; j <= n + 1; ++j) right.push_back(j);

  // conditions (rows) and right-hand sides (one column per node j)
  std::vector<std::vector<Q>> A, B;
  auto add_condition = [&](std::vector<Q> row, std::vector<Q> rhs) {
    A.push_back(row);
    B.push_back(rhs);
  };
  std::vector<Q> e0(I), e1(I);
  for (int c = 0; c < I; ++c) {
    e0[c] = make(all[c] == 0 ? 1 : 0);
    e1[c] = make(all[c] == 1 ? 1 : 0);
  }
  add_condition(functional_row(deg, 0, 0), e0);
  add_condition(functional_row(deg, 0, 1), e1);
  for (int k = 1; k <= m; ++k) {
    std::vector<Q> r0(I), r1(I);
    for (int c = 0; c < I; ++c) {
      int j = all[c];
      bool inl = j <= n, inr = j >= 1 - n;
      r0[c] = inl ? deriv_at(lagrange_basis(left, j), k, 0) : make(0);
      r1[c] = inr ? deriv_at(lagrange_basis(right, j), k, 1) : make(0);
    }
    add_condition(functional_row(deg, k, 0), r0);
    add_condition(functional_row(deg, k, 1), r1);
  }
  for (int r = -(n - m); r <= -1; ++r) {
    std::vector<Q> rr(I);
    for (int c = 0; c < I; ++c) rr[c] = make(all[c] == r ? 1 : 0);
    add_condition(functional_row(deg, 0, r), rr);
  }
  for (int r = 2; r <= n - m + 1; ++r) {
    std::vector<Q> rr(I);
    for (int c = 0; c < I; ++c) rr[c] = make(all[c] == r ? 1 : 0);
    add_condition(functional_row(deg, 0, r), rr);
  }
  if ((int)A.size() != I) return -1;
  if (!solve(A, B)) return -1;
  // B[p][c] is now the coefficient of t^p of beta for node c
  out->I = I;
  for (int c = 0; c < kMaxI; ++c)
    for (int p = 0; p < kMaxI; ++p) {
      out->val64[c][p] = 0.0;
      out->der64[c][p] = 0.0;
      out->val32[c][p] = 0.f;
      out->der32[c][p] = 0.f;
      out->cval64[c][p] = 0.0;
      out->cder64[c][p] = 0.0;
      out->cval32[c][p] = 0.f;
      out->cder32[c][p] = 0.f;
    }
  for (int c = 0; c < I; ++c) {
    Poly mono(I), cen;
    for (int p = 0; p < I; ++p) mono[p] = B[p][c];
    cen = centred(mono);
    for (int p = 0; p < I; ++p) {
      const Q v = mono[p], w = cen[p];
      if (!to_double(v, &out->val64[c][p]) || !to_float(v, &out->val32[c][p])) return -1;
      if (!to_double(w, &out->cval64[c][p]) || !to_float(w, &out->cval32[c][p])) return -1;
      if (p >= 1) {
        const Q d = v * make(p), e = w * make(p);
        if (!to_double(d, &out->der64[c][p - 1]) || !to_float(d, &out->der32[c][p - 1])) return -1;
        if (!to_double(e, &out->cder64[c][p - 1]) || !to_float(e, &out->cder32[c][p - 1])) return -1;
      }
    }
  }
  return g_overflow ? -1 : 0;
}

}  // namespace ptk
