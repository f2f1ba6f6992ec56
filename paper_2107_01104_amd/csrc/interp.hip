// Interpolation of the stored field at binned particles: the weighted triple
// sum of Sec. 2.2, Eq. "triple_sum", and the gradient through derivative
// kernels.
//
// One workgroup per bin (a brick of B^3 cells).  The workgroup first copies
// the brick's halo -- the (B+I-1)^3 nodes any particle of the brick can touch
// -- from the padded field into LDS, converting 3-component nodes to a 4-wide,
// 16-byte-aligned (FP32) / 32-byte (FP64) / 8-byte (BF16, FP16) LDS layout.
// Then each group of GS lanes (GS = 8 for I = 6, 8; 4 for I = 4) takes one
// particle: lane j owns the x1 node offset j and contracts x2 then x3 for the
// three components,
//     s_a(i3) = sum_i2 beta_i2(t2) u_a(c1+j, c2+i2, c3+i3)
//     r_a     = beta_j(t1) * sum_i3 beta_i3(t3) s_a(i3),
// and the group reduces r_a over its lanes (the x1 sum).  This is the paper's
// split of the triple sum into partial sums over some directions finished
// along the remaining one (Sec. 3.3, "split into I double sums"), done inside
// one wavefront instead of across processes.  The eight lanes of a group read
// eight consecutive LDS nodes per (i2, i3), i.e. 128 contiguous bytes.
//
// Weights are evaluated per lane by Horner from the lane's own row of the
// coefficient table and shared in the group with cross-lane reads.
// Sums are FP64 for FP64 storage and FP32 otherwise.  Workgroup-to-bin mapping
// is XCD-aware: consecutive workgroups go round-robin to the 8 XCDs, so each
// XCD is given a contiguous run of bins and neighbouring bricks share its L2.
#include "device_common.h"
#include "launch.h"
#include "ptk_internal.h"

namespace ptk {

enum { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2, ST_F16 = 3 };

template <int ST>
struct StoreT;
template <>
struct StoreT<ST_F64> {
  using acc = double;
  static constexpr int lds_bytes = 32, glob_bytes = 24, G = 2;
};
template <>
struct StoreT<ST_F32> {
  using acc = float;
  static constexpr int lds_bytes = 16, glob_bytes = 12, G = 4;
};
template <>
struct StoreT<ST_BF16> {
  using acc = float;
  static constexpr int lds_bytes = 8, glob_bytes = 6, G = 8;
};
template <>
struct StoreT<ST_F16> {
  using acc = float;
  static constexpr int lds_bytes = 8, glob_bytes = 6, G = 8;
};

// write node q of a 48-byte global chunk (12 words) into LDS node slot n
template <int ST>
__device__ __forceinline__ void lds_put(unsigned char* smem, int n, const uint32_t* w, int q) {
  if constexpr (ST == ST_F32) {
    ((uint4*)smem)[n] = make_uint4(w[3 * q], w[3 * q + 1], w[3 * q + 2], 0u);
  } else if constexpr (ST == ST_F64) {
    ((uint4*)smem)[2 * n] = make_uint4(w[6 * q], w[6 * q + 1], w[6 * q + 2], w[6 * q + 3]);
    ((uint4*)smem)[2 * n + 1] = make_uint4(w[6 * q + 4], w[6 * q + 5], 0u, 0u);
  } else {
    const int k = 3 * q;
    uint32_t h0 = (w[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu;
    uint32_t h1 = (w[(k + 1) >> 1] >> (((k + 1) & 1) * 16)) & 0xFFFFu;
    uint32_t h2 = (w[(k + 2) >> 1] >> (((k + 2) & 1) * 16)) & 0xFFFFu;
    ((uint2*)smem)[n] = make_uint2(h0 | (h1 << 16), h2);
  }
}

template <int ST>
__device__ __forceinline__ void lds_get(const unsigned char* smem, int n, typename StoreT<ST>::acc* v) {
  if constexpr (ST == ST_F32) {
    float4 f = ((const float4*)smem)[n];
    v[0] = f.x;
    v[1] = f.y;
    v[2] = f.z;
  } else if constexpr (ST == ST_F64) {
    double2 a = ((const double2*)smem)[2 * n];
    double2 b = ((const double2*)smem)[2 * n + 1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
  } else if constexpr (ST == ST_BF16) {
    uint2 u = ((const uint2*)smem)[n];
    v[0] = __uint_as_float(u.x << 16);
    v[1] = __uint_as_float(u.x & 0xFFFF0000u);
    v[2] = __uint_as_float(u.y << 16);
  } else {
    uint2 u = ((const uint2*)smem)[n];
    v[0] = __half2float(__ushort_as_half((unsigned short)(u.x & 0xFFFFu)));
    v[1] = __half2float(__ushort_as_half((unsigned short)(u.x >> 16)));
    v[2] = __half2float(__ushort_as_half((unsigned short)(u.y & 0xFFFFu)));
  }
}

template <int I, typename T>
__device__ __forceinline__ T horner(const T* c, T t) {
  T acc = c[I - 1];
#pragma unroll
  for (int p = I - 2; p >= 0; --p) acc = fma(acc, t, c[p]);
  return acc;
}

template <int ST, int I, bool GRAD>
__global__ __launch_bounds__(256) void k_interp(InterpArgs a, int64_t per_xcd) {
  using T = typename StoreT<ST>::acc;
  constexpr int B = kBinEdge;
  constexpr int BX = B + I - 1;
  constexpr int NODES = BX * BX * BX;
  constexpr int G = StoreT<ST>::G;
  constexpr int RG = (BX + G - 1) / G;   // 48-byte chunks per box row
  constexpr int GS = (I <= 4) ? 4 : 8;   // lanes per particle
  constexpr int GPB = 256 / GS;          // particles per workgroup round
  __shared__ __attribute__((aligned(16))) unsigned char smem[NODES * StoreT<ST>::lds_bytes];

  const int64_t bid = blockIdx.x;
  const int64_t bin = (bid & 7) * per_xcd + (bid >> 3);
  if (bin >= a.n_bins) return;
  const uint32_t start = a.offsets[bin], end = a.offsets[bin + 1];
  if (start >= end) return;
  const int nb = a.nb;
  const int bx = (int)(bin % nb), by = (int)((bin / nb) % nb), bz = (int)(bin / ((int64_t)nb * nb));

  // ---- stage the halo brick: box node (z, y, x) = padded node (bz*B+z, by*B+y, bx*B+x)
  {
    const unsigned char* f = (const unsigned char*)a.field;
    const int64_t P = a.P;
    const int64_t x0 = (int64_t)bx * B;
    for (int it = threadIdx.x; it < BX * BX * RG; it += 256) {
      const int g = it % RG;
      const int y = (it / RG) % BX;
      const int z = it / (RG * BX);
      const int64_t Z = (int64_t)bz * B + z, Y = (int64_t)by * B + y;
      const int xs = g * G;
      if (Z >= P || Y >= P || x0 + xs >= P) continue;
      const uint4* src = (const uint4*)(f + Z * a.plane_pitch + Y * a.row_pitch +
                                        (x0 + xs) * StoreT<ST>::glob_bytes);
      uint32_t w[12];
      uint4 c0 = src[0], c1 = src[1], c2 = src[2];
      w[0] = c0.x; w[1] = c0.y; w[2] = c0.z; w[3] = c0.w;
      w[4] = c1.x; w[5] = c1.y; w[6] = c1.z; w[7] = c1.w;
      w[8] = c2.x; w[9] = c2.y; w[10] = c2.z; w[11] = c2.w;
      const int rowbase = (z * BX + y) * BX;
#pragma unroll
      for (int q = 0; q < G; ++q)
        if (xs + q < BX) lds_put<ST>(smem, rowbase + xs + q, w, q);
    }
  }
  __syncthreads();

  // ---- per-lane constants
  const int lane = threadIdx.x & 63;
  const int j = threadIdx.x % GS;            // x1 node offset owned by this lane
  const int jj = j < I ? j : I - 1;          // clamped for the idle lanes of I = 6
  const int gbase = lane - j;                // first lane of this group in the wave
  const int grp = threadIdx.x / GS;
  const KernelTables* tab = (const KernelTables*)a.coef;
  T cv[I], cd[I];
#pragma unroll
  for (int p = 0; p < I; ++p) {
    if constexpr (sizeof(T) == 8) {
      cv[p] = tab->val64[jj][p];
      cd[p] = tab->der64[jj][p];
    } else {
      cv[p] = tab->val32[jj][p];
      cd[p] = tab->der32[jj][p];
    }
  }
  const int N = a.N;
  const double invd = a.invd;
  const int ox = bx * B, oy = by * B, oz = bz * B;

  for (uint32_t p0 = start; p0 < end; p0 += GPB) {
    const uint32_t p = p0 + grp;
    const bool active = p < end;
    const uint32_t pl = active ? p : end - 1;
    // lanes 0, 1, 2 of the group locate axes x1, x2, x3
    const int ax = j < 3 ? j : 2;
    int c;
    double td;
    locate(a.X[3 * (int64_t)pl + ax], N, invd, &c, &td);
    const int c1 = __shfl(c, gbase + 0, 64), c2 = __shfl(c, gbase + 1, 64), c3 = __shfl(c, gbase + 2, 64);
    const double t1d = __shfl(td, gbase + 0, 64), t2d = __shfl(td, gbase + 1, 64),
                 t3d = __shfl(td, gbase + 2, 64);
    const T t1 = (T)t1d, t2 = (T)t2d, t3 = (T)t3d;
    // local cell inside the brick (clamped: the LDS index stays in the box)
    const int l1 = min(max(c1 - ox, 0), B - 1), l2 = min(max(c2 - oy, 0), B - 1),
              l3 = min(max(c3 - oz, 0), B - 1);
    // weights: lane evaluates node jj on every axis, then the group shares x2/x3
    T w1 = horner<I>(cv, t1);
    const T w2j = horner<I>(cv, t2), w3j = horner<I>(cv, t3);
    if (j >= I) w1 = (T)0;
    T w2[I], w3[I];
#pragma unroll
    for (int k = 0; k < I; ++k) {
      w2[k] = __shfl(w2j, gbase + k, 64);
      w3[k] = __shfl(w3j, gbase + k, 64);
    }
    T d1 = 0, dw2[I], dw3[I];
    if constexpr (GRAD) {
      d1 = horner<I - 1>(cd, t1);
      const T d2j = horner<I - 1>(cd, t2), d3j = horner<I - 1>(cd, t3);
      if (j >= I) d1 = (T)0;
#pragma unroll
      for (int k = 0; k < I; ++k) {
        dw2[k] = __shfl(d2j, gbase + k, 64);
        dw3[k] = __shfl(d3j, gbase + k, 64);
      }
    }
    // contraction over x2 then x3 for this lane's x1 node
    const int nbase = (l3 * BX + l2) * BX + l1 + jj;
    T acc[3] = {0, 0, 0}, ad2[3] = {0, 0, 0}, ad3[3] = {0, 0, 0};
#pragma unroll
    for (int i3 = 0; i3 < I; ++i3) {
      T s[3] = {0, 0, 0}, sd[3] = {0, 0, 0};
#pragma unroll
      for (int i2 = 0; i2 < I; ++i2) {
        T v[3];
        lds_get<ST>(smem, nbase + (i3 * BX + i2) * BX, v);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          s[q] = fma(w2[i2], v[q], s[q]);
          if constexpr (GRAD) sd[q] = fma(dw2[i2], v[q], sd[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        acc[q] = fma(w3[i3], s[q], acc[q]);
        if constexpr (GRAD) {
          ad3[q] = fma(dw3[i3], s[q], ad3[q]);
          ad2[q] = fma(w3[i3], sd[q], ad2[q]);
        }
      }
    }
    // x1 weight, then the sum over the group's lanes
    constexpr int NV = GRAD ? 12 : 3;
    T r[NV];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      r[q] = w1 * acc[q];
      if constexpr (GRAD) {
        r[3 + 3 * q + 0] = d1 * acc[q];
        r[3 + 3 * q + 1] = w1 * ad2[q];
        r[3 + 3 * q + 2] = w1 * ad3[q];
      }
    }
#pragma unroll
    for (int o = 1; o < GS; o <<= 1)
#pragma unroll
      for (int e = 0; e < NV; ++e) r[e] += __shfl_xor(r[e], o, 64);
    if (active) {
      const int64_t q = a.orig ? (int64_t)a.orig[p] : (int64_t)p;
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        if (e % GS != j) continue;
        if (e < 3) {
          if (!a.out) continue;
          T val = r[e];
          if constexpr (ST == ST_BF16 || ST == ST_F16) val *= a.scale[e];
          if (a.out_f64)
            ((double*)a.out)[3 * q + e] = (double)val;
          else
            ((float*)a.out)[3 * q + e] = (float)val;
        } else {
          const int comp = (e - 3) / 3;
          T val = r[e] * (T)invd;
          if constexpr (ST == ST_BF16 || ST == ST_F16) val *= a.scale[comp];
          if (a.out_f64)
            ((double*)a.grad)[9 * q + (e - 3)] = (double)val;
          else
            ((float*)a.grad)[9 * q + (e - 3)] = (float)val;
        }
      }
    }
  }
}

template <int ST, int I>
static hipError_t launch_one(const InterpArgs& a, hipStream_t s) {
  const int64_t per_xcd = (a.n_bins + 7) / 8;
  const int64_t grid = per_xcd * 8;
  if (grid == 0) return hipSuccess;
  if (a.grad)
    k_interp<ST, I, true><<<(unsigned)grid, 256, 0, s>>>(a, per_xcd);
  else
    k_interp<ST, I, false><<<(unsigned)grid, 256, 0, s>>>(a, per_xcd);
  return hipGetLastError();
}

template <int ST>
static hipError_t launch_st(int I, const InterpArgs& a, hipStream_t s) {
  switch (I) {
    case 4: return launch_one<ST, 4>(a, s);
    case 6: return launch_one<ST, 6>(a, s);
    case 8: return launch_one<ST, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_interp(int storage, int I, const InterpArgs& a, hipStream_t s) {
  switch (storage) {
    case ST_F64: return launch_st<ST_F64>(I, a, s);
    case ST_F32: return launch_st<ST_F32>(I, a, s);
    case ST_BF16: return launch_st<ST_BF16>(I, a, s);
    case ST_F16: return launch_st<ST_F16>(I, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptk
