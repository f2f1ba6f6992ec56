// Field set-up: per-component sum of squares (for the BF16/FP16 scale) and the
// copy of a grid field into the stored layout, and the copy back out.  The
// source is described by element strides (SrcLayout): the caller's
// u[x3][x2][x1][3], or the three padded real planes an inverse transform
// leaves.
//
// Stored layout: the periodic field padded by I/2-1 nodes below and I/2 nodes
// above on every axis (so every stencil c + i, i = 1-I/2..I/2, of Eq.
// "triple_sum" is a plain box without modulo arithmetic), 3 components per
// node in the storage type, x1 rows padded to a 64-byte multiple with at
// least 48 spare bytes (the interpolation kernel reads rows in 48-byte chunks).
#include "device_common.h"
#include "launch.h"

namespace ptk {

// node (x1, x2, x3) of the source, component 0
__device__ __forceinline__ int64_t src_node(const SrcLayout& l, int64_t x1, int64_t x2, int64_t x3) {
  return x3 * l.ps + x2 * l.rs + x1 * l.ns;
}

__global__ __launch_bounds__(256) void k_sumsq(const void* __restrict__ u, int in_f64, int64_t N, SrcLayout l,
                                               double* __restrict__ partial) {
  __shared__ double sh[3][256];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const int64_t nodes = N * N * N;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nodes; i += (int64_t)gridDim.x * 256) {
    const int64_t o = src_node(l, i % N, (i / N) % N, i / (N * N));
    double a, b, c;
    if (in_f64) {
      const double* d = (const double*)u;
      a = d[o];
      b = d[o + l.cs];
      c = d[o + 2 * l.cs];
    } else {
      const float* f = (const float*)u;
      a = f[o];
      b = f[o + l.cs];
      c = f[o + 2 * l.cs];
    }
    s0 += a * a;
    s1 += b * b;
    s2 += c * c;
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 3) partial[3 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_sumsq(const void* u, int in_f64, int64_t N, const SrcLayout& l, double* partial, int nblocks,
                        hipStream_t s) {
  k_sumsq<<<nblocks, 256, 0, s>>>(u, in_f64, N, l, partial);
  return hipGetLastError();
}

// padded index k (0 <= k < N + I - 1) holds grid node (k - halo_lo) mod N
__device__ __forceinline__ int wrap_node(int k, int halo_lo, int N) {
  const int j = k - halo_lo;
  return j < 0 ? j + N : (j >= N ? j - N : j);
}

// One padded plane z per blockIdx.y, its P*P nodes over blockIdx.x (32-bit
// index arithmetic: P <= 4103, so P*P < 2^25)
template <int STORAGE>
__global__ __launch_bounds__(256) void k_pack(const void* __restrict__ u, int in_f64, SrcLayout l, int N, int P,
                                              int halo_lo, unsigned char* __restrict__ field, int64_t row_pitch,
                                              int64_t plane_pitch, float inv0, float inv1, float inv2) {
  const int z = blockIdx.y;
  const uint32_t yx = blockIdx.x * 256u + threadIdx.x;
  if (yx >= (uint32_t)(P * P)) return;
  const int y = (int)(yx / (uint32_t)P), x = (int)yx - y * P;
  const int64_t src = src_node(l, wrap_node(x, halo_lo, N), wrap_node(y, halo_lo, N), wrap_node(z, halo_lo, N));
  double v[3];
  for (int q = 0; q < 3; ++q)
    v[q] = in_f64 ? ((const double*)u)[src + q * l.cs] : (double)((const float*)u)[src + q * l.cs];
  unsigned char* dst = field + z * plane_pitch + y * row_pitch;
  if constexpr (STORAGE == 0) {
    double* d = (double*)(dst + x * 24);
    d[0] = v[0];
    d[1] = v[1];
    d[2] = v[2];
  } else if constexpr (STORAGE == 1) {
    float* d = (float*)(dst + x * 12);
    d[0] = (float)v[0];
    d[1] = (float)v[1];
    d[2] = (float)v[2];
  } else {
    // fl32(u32 * fl32(1/s_a)), then round to nearest even in 16 bits
    const float inv[3] = {inv0, inv1, inv2};
    uint16_t* d = (uint16_t*)(dst + x * 6);
    for (int q = 0; q < 3; ++q) {
      float sc = (float)v[q] * inv[q];
      if constexpr (STORAGE == 2)
        d[q] = f32_to_bf16_rne(sc);
      else
        d[q] = f32_to_f16_rne(sc);
    }
  }
}

hipError_t launch_pack(const void* u, int in_f64, const SrcLayout& l, int64_t N, int storage, int I, void* field,
                       int64_t row_pitch, int64_t plane_pitch, const float* inv_scale, hipStream_t s) {
  const int P = (int)(N + I - 1);
  const int halo_lo = I / 2 - 1;
  const dim3 grid((unsigned)(((int64_t)P * P + 255) / 256), (unsigned)P);
  unsigned char* f = (unsigned char*)field;
  const float i0 = inv_scale[0], i1 = inv_scale[1], i2 = inv_scale[2];
  const int n = (int)N;
  switch (storage) {
    case 0: k_pack<0><<<grid, 256, 0, s>>>(u, in_f64, l, n, P, halo_lo, f, row_pitch, plane_pitch, i0, i1, i2); break;
    case 1: k_pack<1><<<grid, 256, 0, s>>>(u, in_f64, l, n, P, halo_lo, f, row_pitch, plane_pitch, i0, i1, i2); break;
    case 2: k_pack<2><<<grid, 256, 0, s>>>(u, in_f64, l, n, P, halo_lo, f, row_pitch, plane_pitch, i0, i1, i2); break;
    case 3: k_pack<3><<<grid, 256, 0, s>>>(u, in_f64, l, n, P, halo_lo, f, row_pitch, plane_pitch, i0, i1, i2); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The stored field without its halo, as out[x3][x2][x1][3]: stored values
// converted exactly (16-bit codes stay unscaled).
template <int STORAGE, typename O>
__global__ __launch_bounds__(256) void k_unpack(const unsigned char* __restrict__ field, int N, int halo_lo,
                                                int64_t row_pitch, int64_t plane_pitch, O* __restrict__ out) {
  const int z = blockIdx.y;
  const uint32_t yx = blockIdx.x * 256u + threadIdx.x;
  if (yx >= (uint32_t)(N * N)) return;
  const int y = (int)(yx / (uint32_t)N), x = (int)yx - y * N;
  const unsigned char* src = field + (int64_t)(z + halo_lo) * plane_pitch + (int64_t)(y + halo_lo) * row_pitch;
  const int xs = x + halo_lo;
  const int64_t i = (int64_t)z * N * N + yx;
  for (int q = 0; q < 3; ++q) {
    O v;
    if constexpr (STORAGE == 0) {
      v = (O)((const double*)(src + xs * 24))[q];
    } else if constexpr (STORAGE == 1) {
      v = (O)((const float*)(src + xs * 12))[q];
    } else {
      const uint16_t b = ((const uint16_t*)(src + xs * 6))[q];
      if constexpr (STORAGE == 2)
        v = (O)bf16_to_f32(b);
      else
        v = (O)__half2float(__ushort_as_half((unsigned short)b));
    }
    out[3 * i + q] = v;
  }
}

hipError_t launch_unpack(const void* field, int64_t N, int storage, int I, int64_t row_pitch, int64_t plane_pitch,
                         void* out, int out_f64, hipStream_t s) {
  const int n = (int)N;
  const dim3 g((unsigned)(((int64_t)n * n + 255) / 256), (unsigned)n);
  const unsigned char* f = (const unsigned char*)field;
  const int h = I / 2 - 1;
#define PTK_UNPACK(ST)                                                                              \
  if (out_f64)                                                                                       \
    k_unpack<ST, double><<<g, 256, 0, s>>>(f, n, h, row_pitch, plane_pitch, (double*)out);           \
  else                                                                                               \
    k_unpack<ST, float><<<g, 256, 0, s>>>(f, n, h, row_pitch, plane_pitch, (float*)out);
  switch (storage) {
    case 0: PTK_UNPACK(0) break;
    case 1: PTK_UNPACK(1) break;
    case 2: PTK_UNPACK(2) break;
    case 3: PTK_UNPACK(3) break;
    default: return hipErrorInvalidValue;
  }
#undef PTK_UNPACK
  return hipGetLastError();
}

}  // namespace ptk
