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

template <typename V>
__global__ __launch_bounds__(256) void k_update(int kind, const double* __restrict__ X, UpdateVel v, double dt,
                                                int64_t n, double* __restrict__ Xout, uint32_t* __restrict__ keys,
                                                int N, double invd, BinGeom g, int* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const V* k0 = (const V*)v.k[0];
  const V* k1 = (const V*)v.k[1];
  const V* k2 = (const V*)v.k[2];
  const V* k3 = (const V*)v.k[3];
  int c[3];
  bool ok = true;
  const double hdt = 0.5 * dt;
  for (int d = 0; d < 3; ++d) {
    const double x = X[3 * i + d];
    const double a = (double)k0[3 * i + d];
    double xn;
    if (kind == kEulerOrPredict) {
      xn = x + dt * a;
    } else if (kind == kHeunCorrect) {
      const double b = (double)k1[3 * i + d];
      xn = x + hdt * (a + b);
    } else {
      double inc = v.b[0] * a;
      if (v.nk > 1) inc = inc + v.b[1] * (double)k1[3 * i + d];
      if (v.nk > 2) inc = inc + v.b[2] * (double)k2[3 * i + d];
      if (v.nk > 3) inc = inc + v.b[3] * (double)k3[3 * i + d];
      xn = x + dt * inc;
    }
    if (!in_domain(xn)) {
      ok = false;
      xn = 0.0;
    }
    double t;
    const double y = locate(xn, N, invd, &c[d], &t);
    Xout[3 * i + d] = y;
  }
  if (!ok) flag[0] = 1;
  keys[i] = bin_key(c[0], c[1], c[2], g);
}

hipError_t launch_update(int kind, int vel_f64, const double* X, const UpdateVel& v, double dt, int64_t n,
                         double* Xout, uint32_t* keys, int N, double invd, const BinGeom& g, int* flag,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (vel_f64)
    k_update<double><<<blocks, 256, 0, s>>>(kind, X, v, dt, n, Xout, keys, N, invd, g, flag);
  else
    k_update<float><<<blocks, 256, 0, s>>>(kind, X, v, dt, n, Xout, keys, N, invd, g, flag);
  return hipGetLastError();
}

}  // namespace ptk
