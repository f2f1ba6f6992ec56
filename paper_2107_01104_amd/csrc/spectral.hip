// Velocity on the grid from the spectral state: the inverse transform that
// particle tracking adds to each step of the pseudo-spectral solver (Sec. 4.2,
// "IFT for PT" of the overall-performance breakdown).
//
// Input: the half spectrum of a real field, N x N x (N/2+1) modes (Sec. 2.1),
// index order [k2][k3][k1][a] -- directions 2 and 3 transposed against the
// grid's [x3][x2][x1], as in the paper's slab layout (Sec. 3.2) -- with
// complex numbers as (re, im) pairs.  Either the velocity amplitudes u^(k), or
// the vorticity w^(k), from which the Biot-Savart law of Sec. 2.1 gives
// u^(k) = i k x w^(k) / |k|^2.
//
// k_spec_prep writes the three components as [a][k3][k2][k1] (one thread per
// mode: coalesced writes, and each thread reads its mode's three components
// from one 48-byte (FP64) or 24-byte (FP32) span); the inverse real transform
// of the three components then runs out of place (rocFFT, batch of 3; about 5%
// faster than in place at 1024^3), leaving three real planes [a][x3][x2][x1]
// that the field pack reads through its strided source layout.
#include <rocfft/rocfft.h>

#include <mutex>
#include <new>

#include "launch.h"

namespace ptk {

// One k3 plane per blockIdx.y, its N (N/2+1) modes over blockIdx.x (32-bit
// index arithmetic within the plane: N <= 2048)
template <typename R>
__global__ __launch_bounds__(256) void k_spec_prep(const R* __restrict__ in, int N, int vorticity,
                                                   R* __restrict__ out) {
  const int H = N / 2 + 1;
  const int64_t modes = (int64_t)N * N * H;
  const int k3 = blockIdx.y;
  const uint32_t r = blockIdx.x * 256u + threadIdx.x;
  if (r < (uint32_t)(N * H)) {
    const int k2 = (int)(r / (uint32_t)H), k1 = (int)r - k2 * H;
    const int64_t i = (int64_t)k3 * N * H + r;  // the mode's index in [k3][k2][k1] order
    const int64_t src = (((int64_t)k2 * N + k3) * H + k1) * 3;
    R re[3], im[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      re[a] = in[2 * (src + a)];
      im[a] = in[2 * (src + a) + 1];
    }
    if (vorticity) {
      // signed wave numbers (index - N above N/2); the Nyquist index N/2 has
      // no sign, and a derivative there has no real representation: zero
      const int n2 = N / 2;
      const bool nyq = k1 == n2 || k2 == n2 || k3 == n2;
      const R q1 = (R)k1, q2 = (R)(k2 <= n2 ? k2 : k2 - N), q3 = (R)(k3 <= n2 ? k3 : k3 - N);
      const R kk = q1 * q1 + q2 * q2 + q3 * q3;
      // c = k x w (k real), then u = i c / |k|^2
      const R cr[3] = {q2 * re[2] - q3 * re[1], q3 * re[0] - q1 * re[2], q1 * re[1] - q2 * re[0]};
      const R ci[3] = {q2 * im[2] - q3 * im[1], q3 * im[0] - q1 * im[2], q1 * im[1] - q2 * im[0]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const bool zero = nyq || kk == (R)0;
        re[a] = zero ? (R)0 : -ci[a] / kk;
        im[a] = zero ? (R)0 : cr[a] / kk;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      out[2 * (a * modes + i)] = re[a];
      out[2 * (a * modes + i) + 1] = im[a];
    }
  }
}

hipError_t launch_spec_prep(const void* spec, int in_f64, int64_t N, int vorticity, void* out, hipStream_t s) {
  const int n = (int)N;
  const dim3 grid((unsigned)(((int64_t)n * (n / 2 + 1) + 255) / 256), (unsigned)n);
  if (in_f64)
    k_spec_prep<double><<<grid, 256, 0, s>>>((const double*)spec, n, vorticity, (double*)out);
  else
    k_spec_prep<float><<<grid, 256, 0, s>>>((const float*)spec, n, vorticity, (float*)out);
  return hipGetLastError();
}

struct FftState {
  rocfft_plan plan = nullptr;
  rocfft_execution_info info = nullptr;
  int64_t N = 0;
  int f64 = -1;
  size_t work = 0;
};

namespace {
std::once_flag g_fft_setup;
rocfft_status g_fft_setup_status = rocfft_status_success;

void destroy_plan(FftState* st) {
  if (st->info) (void)rocfft_execution_info_destroy(st->info);
  if (st->plan) (void)rocfft_plan_destroy(st->plan);
  st->info = nullptr;
  st->plan = nullptr;
  st->N = 0;
  st->f64 = -1;
  st->work = 0;
}
}  // namespace

int fft_prepare(FftState** pst, int64_t N, int f64, size_t* work_bytes, const char** err) {
  std::call_once(g_fft_setup, [] { g_fft_setup_status = rocfft_setup(); });
  if (g_fft_setup_status != rocfft_status_success) {
    *err = "rocfft_setup failed";
    return -1;
  }
  if (!*pst) {
    *pst = new (std::nothrow) FftState();
    if (!*pst) {
      *err = "host allocation failed";
      return -1;
    }
  }
  FftState* st = *pst;
  if (st->plan && st->N == N && st->f64 == f64) {
    *work_bytes = st->work;
    return 0;
  }
  destroy_plan(st);
  const size_t n = (size_t)N, h = n / 2 + 1;
  // element strides, x1 first: hermitian input (complex elements), real
  // output to a separate buffer (unpadded planes); batch distance one component
  const size_t in_strides[3] = {1, h, h * n};
  const size_t out_strides[3] = {1, n, n * n};
  const size_t lengths[3] = {n, n, n};
  rocfft_plan_description desc = nullptr;
  if (rocfft_plan_description_create(&desc) != rocfft_status_success) {
    *err = "rocfft_plan_description_create failed";
    return -1;
  }
  rocfft_status r = rocfft_plan_description_set_data_layout(
      desc, rocfft_array_type_hermitian_interleaved, rocfft_array_type_real, nullptr, nullptr, 3, in_strides,
      h * n * n, 3, out_strides, n * n * n);
  if (r == rocfft_status_success)
    r = rocfft_plan_create(&st->plan, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                           f64 ? rocfft_precision_double : rocfft_precision_single, 3, lengths, 3, desc);
  (void)rocfft_plan_description_destroy(desc);
  if (r != rocfft_status_success) {
    st->plan = nullptr;
    *err = "rocfft_plan_create failed";
    return -1;
  }
  if (rocfft_plan_get_work_buffer_size(st->plan, &st->work) != rocfft_status_success ||
      rocfft_execution_info_create(&st->info) != rocfft_status_success) {
    destroy_plan(st);
    *err = "rocfft plan set-up failed";
    return -1;
  }
  st->N = N;
  st->f64 = f64;
  *work_bytes = st->work;
  return 0;
}

int fft_run(FftState* st, void* buf, void* out, void* work, size_t work_bytes, hipStream_t s, const char** err) {
  if (!st || !st->plan) {
    *err = "no transform plan";
    return -1;
  }
  if (rocfft_execution_info_set_stream(st->info, (void*)s) != rocfft_status_success) {
    *err = "rocfft_execution_info_set_stream failed";
    return -1;
  }
  if (st->work > 0 &&
      rocfft_execution_info_set_work_buffer(st->info, work, work_bytes) != rocfft_status_success) {
    *err = "rocfft_execution_info_set_work_buffer failed";
    return -1;
  }
  void* in[1] = {buf};
  void* outs[1] = {out};
  if (rocfft_execute(st->plan, in, outs, st->info) != rocfft_status_success) {
    *err = "rocfft_execute failed";
    return -1;
  }
  return 0;
}

void fft_release(FftState* st) {
  if (!st) return;
  destroy_plan(st);
  delete st;
}

}  // namespace ptk
