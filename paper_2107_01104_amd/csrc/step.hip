// Position updates of the tracer ODE dX/dt = u(X) (Eq. "tracers"), fused with
// the bin key of the new position so that the next re-binning needs no
// separate key pass.  The state is the position itself, not wrapped: the
// reduction modulo 2*pi is step 1 of every interpolation (Sec. 2.2), here only
// inside the key's cell location, so trajectories keep their crossings of
// the periodic faces.  Velocities come in as FP64 or FP32
// and are widened to FP64; every operation is a separately rounded binary64
// operation in the order written (the file is built with -ffp-contract=off).
//   kEulerOrPredict: X + dt*k0              (Euler step, Heun predictor)
//   kHeunCorrect:    X + (0.5*dt)*(k0 + k1) (Heun corrector)
//   kAB:             X + dt*(b0*k0 + b1*k1 + ...), k_j = u_{n-j}, the
//                    Adams-Bashforth weights of the step's order (2..4)
#include "device_common.h"
#include "launch.h"

namespace ptk {

// One block: 512 particles, 256 threads.  Positions and velocities are [n][3]
// rows; the block stages its consecutive rows of each through LDS (16-byte
// loads and stores where the block is full and the arrays are 16-byte
// aligned), so every global access is a unit-stride wave access, then each
// thread updates two particles.  Positions may be read through a row index
// (xrow): consecutive threads then read the coordinates of the rows in turn,
// which stays nearly unit-stride while the index is close to the identity (a
// re-binning after one time step).
constexpr int kUpdThreads = 256;
constexpr int kUpdParts = 512;

template <typename V>
__device__ __forceinline__ void stage_in(void* dst, const void* src, int nbytes, bool vec) {
  if (vec) {
    for (int e = threadIdx.x; e < nbytes / 16; e += kUpdThreads) ((uint4*)dst)[e] = ((const uint4*)src)[e];
  } else {
    for (int e = threadIdx.x; e < nbytes / (int)sizeof(V); e += kUpdThreads) ((V*)dst)[e] = ((const V*)src)[e];
  }
}

template <typename V>
__global__ __launch_bounds__(kUpdThreads) void k_update(int kind, const double* __restrict__ X,
                                                        const uint32_t* __restrict__ xrow, UpdateVel v,
                                                        double dt, int64_t n, double* __restrict__ Xout,
                                                        uint32_t* __restrict__ keys, int N, double invd, BinGeom g,
                                                        int* __restrict__ flag, int aligned) {
  extern __shared__ __attribute__((aligned(16))) unsigned char upd_smem[];
  double* sx = (double*)upd_smem;                         // [3 * kUpdParts]
  V* sk = (V*)(upd_smem + 3 * kUpdParts * sizeof(double));  // [nk][3 * kUpdParts]
  const int64_t base = (int64_t)blockIdx.x * kUpdParts;
  const int nb = (int)min((int64_t)kUpdParts, n - base);
  const int nk = kind == kEulerOrPredict ? 1 : kind == kHeunCorrect ? 2 : v.nk;
  const bool vec = aligned && nb == kUpdParts;
  if (xrow) {
    // each thread's two particles: both row indices, then all six
    // coordinates, so the loads are in flight together
    static_assert(kUpdParts == 2 * kUpdThreads, "two particles per thread");
    const int p0 = threadIdx.x, p1 = threadIdx.x + kUpdThreads;
    const int64_t r0 = p0 < nb ? (int64_t)xrow[base + p0] : 0;
    const int64_t r1 = p1 < nb ? (int64_t)xrow[base + p1] : 0;
    double c0[3], c1[3];
    for (int d = 0; d < 3; ++d) {
      c0[d] = p0 < nb ? X[3 * r0 + d] : 0.0;
      c1[d] = p1 < nb ? X[3 * r1 + d] : 0.0;
    }
    for (int d = 0; d < 3; ++d) {
      if (p0 < nb) sx[3 * p0 + d] = c0[d];
      if (p1 < nb) sx[3 * p1 + d] = c1[d];
    }
  } else {
    stage_in<double>(sx, X + 3 * base, 3 * nb * (int)sizeof(double), vec);
  }
  for (int j = 0; j < nk; ++j)
    stage_in<V>(sk + j * 3 * kUpdParts, (const V*)v.k[j] + 3 * base, 3 * nb * (int)sizeof(V), vec);
  __syncthreads();
  const double hdt = 0.5 * dt;
  for (int p = threadIdx.x; p < nb; p += kUpdThreads) {
    int c[3];
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
      const int e = 3 * p + d;
      const double x = sx[e];
      const double a = (double)sk[e];
      double xn;
      if (kind == kEulerOrPredict) {
        xn = x + dt * a;
      } else if (kind == kHeunCorrect) {
        const double b = (double)sk[3 * kUpdParts + e];
        xn = x + hdt * (a + b);
      } else {
        double inc = v.b[0] * a;
        if (nk > 1) inc = inc + v.b[1] * (double)sk[3 * kUpdParts + e];
        if (nk > 2) inc = inc + v.b[2] * (double)sk[6 * kUpdParts + e];
        if (nk > 3) inc = inc + v.b[3] * (double)sk[9 * kUpdParts + e];
        xn = x + dt * inc;
      }
      if (!in_domain(xn)) {
        ok = false;
        xn = 0.0;
      }
      double t;
      (void)locate(xn, N, invd, &c[d], &t);
      sx[e] = xn;  // only this thread touches its three entries
    }
    if (!ok) atomicOr(flag, kFlagDomain);
    keys[base + p] = bin_key(c[0], c[1], c[2], g);
  }
  __syncthreads();
  if (vec) {
    for (int e = threadIdx.x; e < 3 * kUpdParts * 8 / 16; e += kUpdThreads)
      ((uint4*)(Xout + 3 * base))[e] = ((const uint4*)sx)[e];
  } else {
    for (int e = threadIdx.x; e < 3 * nb; e += kUpdThreads) Xout[3 * base + e] = sx[e];
  }
}

hipError_t launch_update(int kind, int vel_f64, const double* X, const uint32_t* xrow, const UpdateVel& v, double dt,
                         int64_t n, double* Xout, uint32_t* keys, int N, double invd, const BinGeom& g, int* flag,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nk = kind == kEulerOrPredict ? 1 : kind == kHeunCorrect ? 2 : v.nk;
  if (nk < 1 || nk > 4) return hipErrorInvalidValue;
  for (int j = 0; j < nk; ++j)
    if (!v.k[j]) return hipErrorInvalidValue;
  bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)Xout % 16 == 0);
  for (int j = 0; j < nk; ++j) aligned = aligned && ((uintptr_t)v.k[j] % 16 == 0);
  const unsigned blocks = (unsigned)((n + kUpdParts - 1) / kUpdParts);
  const size_t vb = vel_f64 ? sizeof(double) : sizeof(float);
  const size_t lds = 3 * kUpdParts * sizeof(double) + (size_t)nk * 3 * kUpdParts * vb;
  if (vel_f64)
    k_update<double><<<blocks, kUpdThreads, lds, s>>>(kind, X, xrow, v, dt, n, Xout, keys, N, invd, g, flag,
                                                       aligned);
  else
    k_update<float><<<blocks, kUpdThreads, lds, s>>>(kind, X, xrow, v, dt, n, Xout, keys, N, invd, g, flag,
                                                      aligned);
  return hipGetLastError();
}

// ---- Orientation of axisymmetric ellipsoids (Jeffery's equation):
//   dp/dt = W p + shape (S p - (p . S p) p),  S = (A + A^T)/2, W = (A - A^T)/2,
// A[a][b] = du_a/dx_b the interpolated gradient (FP64 or FP32, widened).
// Every operation is a separately rounded binary64 operation.

template <typename V>
__global__ __launch_bounds__(256) void k_jeffery_rhs(const V* __restrict__ G, const double* __restrict__ p,
                                                     double shape, int64_t n, double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double A[3][3], q[3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A[a][b] = (double)G[9 * i + 3 * a + b];
  for (int a = 0; a < 3; ++a) q[a] = p[3 * i + a];
  double Sp[3], Wp[3];
  for (int a = 0; a < 3; ++a) {
    double s = 0.0, w = 0.0;
    for (int b = 0; b < 3; ++b) {
      const double sab = 0.5 * (A[a][b] + A[b][a]);
      const double wab = 0.5 * (A[a][b] - A[b][a]);
      s = s + sab * q[b];
      w = w + wab * q[b];
    }
    Sp[a] = s;
    Wp[a] = w;
  }
  const double pSp = (q[0] * Sp[0] + q[1] * Sp[1]) + q[2] * Sp[2];
  for (int a = 0; a < 3; ++a) r[3 * i + a] = Wp[a] + shape * (Sp[a] - pSp * q[a]);
}

// p_out = p + dt (b0 r0 + b1 r1 + ...), or p + (0.5 dt)(r0 + r1) for the Heun
// corrector, then (with `unit`) divided by its length.
__global__ __launch_bounds__(256) void k_orient_update(int kind, const double* __restrict__ p, UpdateVel v,
                                                       double dt, int64_t n, int unit, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int nk = kind == kEulerOrPredict ? 1 : kind == kHeunCorrect ? 2 : v.nk;
  double q[3];
  for (int d = 0; d < 3; ++d) {
    const int64_t e = 3 * i + d;
    const double a = ((const double*)v.k[0])[e];
    double x;
    if (kind == kEulerOrPredict) {
      x = p[e] + dt * a;
    } else if (kind == kHeunCorrect) {
      x = p[e] + (0.5 * dt) * (a + ((const double*)v.k[1])[e]);
    } else {
      double inc = v.b[0] * a;
      for (int j = 1; j < nk; ++j) inc = inc + v.b[j] * ((const double*)v.k[j])[e];
      x = p[e] + dt * inc;
    }
    q[d] = x;
  }
  if (unit) {
    const double len = sqrt((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]);
    for (int d = 0; d < 3; ++d) q[d] = q[d] / len;
  }
  for (int d = 0; d < 3; ++d) out[3 * i + d] = q[d];
}

hipError_t launch_jeffery_rhs(int grad_f64, const void* G, const double* p, double shape, int64_t n, double* r,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (grad_f64)
    k_jeffery_rhs<double><<<blocks, 256, 0, s>>>((const double*)G, p, shape, n, r);
  else
    k_jeffery_rhs<float><<<blocks, 256, 0, s>>>((const float*)G, p, shape, n, r);
  return hipGetLastError();
}

// Drag on inertial particles: r = (u - V) / tau per component, FP64 (u in
// the interpolation's precision, converted exactly).
template <typename U>
__global__ __launch_bounds__(256) void k_drag_rhs(const U* __restrict__ u, const double* __restrict__ V, double tau,
                                                  int64_t n3, double* __restrict__ r) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n3) return;
  r[e] = ((double)u[e] - V[e]) / tau;
}

hipError_t launch_drag_rhs(int vel_f64, const void* u, const double* V, double tau, int64_t n, double* r,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t n3 = 3 * n;
  const unsigned blocks = (unsigned)((n3 + 255) / 256);
  if (vel_f64)
    k_drag_rhs<double><<<blocks, 256, 0, s>>>((const double*)u, V, tau, n3, r);
  else
    k_drag_rhs<float><<<blocks, 256, 0, s>>>((const float*)u, V, tau, n3, r);
  return hipGetLastError();
}

hipError_t launch_orient_update(int kind, const double* p, const UpdateVel& v, double dt, int64_t n, int unit,
                                double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nk = kind == kEulerOrPredict ? 1 : kind == kHeunCorrect ? 2 : v.nk;
  if (nk < 1 || nk > 4) return hipErrorInvalidValue;
  for (int j = 0; j < nk; ++j)
    if (!v.k[j]) return hipErrorInvalidValue;
  k_orient_update<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(kind, p, v, dt, n, unit, out);
  return hipGetLastError();
}

}  // namespace ptk
