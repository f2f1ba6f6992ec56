// Position updates of the tracer ODE dX/dt = u(X) (Eq. "tracers") with the
// periodic wrap, fused with the bin key of the new position so that the next
// re-binning needs no separate key pass.  Velocities come in as FP64 or FP32
// and are widened to FP64; every operation is a separately rounded binary64
// operation in the order written (the file is built with -ffp-contract=off).
//   kEulerOrPredict: X + dt*k0              (Euler step, Heun predictor)
//   kHeunCorrect:    X + (0.5*dt)*(k0 + k1) (Heun corrector)
//   kAB:             X + dt*(b0*k0 + b1*k1 + ...), k_j = u_{n-j}, the
//                    Adams-Bashforth weights of the step's order (2..4)
#include "device_common.h"
#include "launch.h"

namespace ptk {

// One block: 256 particles.  Positions and velocities are [n][3] rows; the
// block stages its 768 consecutive entries of each through LDS so that every
// global access is a unit-stride wave access, then each thread updates one
// particle.
constexpr int kUpdBlock = 256;
template <typename V>
__global__ __launch_bounds__(kUpdBlock) void k_update(int kind, const double* __restrict__ X, UpdateVel v, double dt,
                                                      int64_t n, double* __restrict__ Xout, uint32_t* __restrict__ keys,
                                                      int N, double invd, BinGeom g, int* __restrict__ flag) {
  __shared__ double sx[3 * kUpdBlock];
  __shared__ V sk[4][3 * kUpdBlock];
  const int64_t base = (int64_t)blockIdx.x * kUpdBlock;
  const int nb = (int)min((int64_t)kUpdBlock, n - base);
  const int ne = 3 * nb;
  const int nk = kind == kEulerOrPredict ? 1 : kind == kHeunCorrect ? 2 : v.nk;
  const int tid = threadIdx.x;
  for (int e = tid; e < ne; e += kUpdBlock) {
    sx[e] = X[3 * base + e];
    for (int j = 0; j < nk; ++j) sk[j][e] = ((const V*)v.k[j])[3 * base + e];
  }
  __syncthreads();
  if (tid < nb) {
    int c[3];
    bool ok = true;
    const double hdt = 0.5 * dt;
    for (int d = 0; d < 3; ++d) {
      const int e = 3 * tid + d;
      const double x = sx[e];
      const double a = (double)sk[0][e];
      double xn;
      if (kind == kEulerOrPredict) {
        xn = x + dt * a;
      } else if (kind == kHeunCorrect) {
        const double b = (double)sk[1][e];
        xn = x + hdt * (a + b);
      } else {
        double inc = v.b[0] * a;
        if (nk > 1) inc = inc + v.b[1] * (double)sk[1][e];
        if (nk > 2) inc = inc + v.b[2] * (double)sk[2][e];
        if (nk > 3) inc = inc + v.b[3] * (double)sk[3][e];
        xn = x + dt * inc;
      }
      if (!in_domain(xn)) {
        ok = false;
        xn = 0.0;
      }
      double t;
      sx[e] = locate(xn, N, invd, &c[d], &t);  // only this thread touches its three entries
    }
    if (!ok) flag[0] = 1;
    keys[base + tid] = bin_key(c[0], c[1], c[2], g);
  }
  __syncthreads();
  for (int e = tid; e < ne; e += kUpdBlock) Xout[3 * base + e] = sx[e];
}

hipError_t launch_update(int kind, int vel_f64, const double* X, const UpdateVel& v, double dt, int64_t n,
                         double* Xout, uint32_t* keys, int N, double invd, const BinGeom& g, int* flag,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (kind == kAB && (v.nk < 1 || v.nk > 4)) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((n + kUpdBlock - 1) / kUpdBlock);
  if (vel_f64)
    k_update<double><<<blocks, kUpdBlock, 0, s>>>(kind, X, v, dt, n, Xout, keys, N, invd, g, flag);
  else
    k_update<float><<<blocks, kUpdBlock, 0, s>>>(kind, X, v, dt, n, Xout, keys, N, invd, g, flag);
  return hipGetLastError();
}

}  // namespace ptk
