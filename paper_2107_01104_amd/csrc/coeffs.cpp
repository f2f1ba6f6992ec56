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

// Correctly rounded conversion of an exact rational: one IEEE division of
// exactly representable operands.
bool to_double(Q q, double* out) {
  const i128 lim = (i128)1 << 53;
  if (iabs(q.num) >= lim || q.den >= lim) return false;
  *out = (double)(int64_t)q.num / (double)(int64_t)q.den;
  return true;
}

bool to_float(Q q, float* out) {
  const i128 lim = (i128)1 << 24;
  if (iabs(q.num) >= lim || q.den >= lim) return false;
  *out = (float)(int32_t)q.num / (float)(int32_t)q.den;
  return true;
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
    }
  for (int c = 0; c < I; ++c) {
    for (int p = 0; p < I; ++p) {
      Q v = B[p][c];
      if (!to_double(v, &out->val64[c][p]) || !to_float(v, &out->val32[c][p])) return -1;
      if (p >= 1) {
        Q d = v * make(p);
        if (!to_double(d, &out->der64[c][p - 1]) || !to_float(d, &out->der32[c][p - 1])) return -1;
      }
    }
  }
  return 0;
}

}  // namespace ptk
