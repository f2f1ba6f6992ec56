// Interpolation of the stored field at binned particles: the weighted triple
// sum of Sec. 2.2, Eq. "triple_sum", and the gradient through derivative
// kernels.
//
// Work decomposition: a workgroup owns one tile column -- T x T cells in
// (x1, x2), a run of x3 -- and sweeps it along x3, the paper's slice
// direction, in windows of W = 5 cell layers.  Particles are binned by (tile,
// window) with x3 fastest, so a window's particles are contiguous.  The
// (T+I-1)^2 halo nodes of the W+I-1 x3 planes a window touches live in an LDS
// ring; each plane is read from HBM once per tile column (halo over-fetch
// ((T+I-1)/T)^2, 2.5 for T = 12, I = 8), and the planes the next windows add
// are loaded into registers while the current window is computed.  With FP32
// and 16-bit nodes the ring leaves room for two 512-thread workgroups per CU
// (16 waves); FP64 nodes fill the LDS with one.
//
// Per particle: a group of 16 lanes (a DPP row).  Lane j = lane & 7 owns the
// x1 node offset j; the two half-rows split the particle's I planes between
// them.  Each lane contracts x2 for each of its planes and x3 over them,
// scales by its x1 weight, and the group sums over its lanes with DPP: the
// paper's split of the triple sum into partial sums finished along the
// remaining direction (Sec. 3.3), inside one wavefront.  Plane pitches are
// 128 mod 256 bytes, so a particle's 16 lanes read 256 consecutive bytes
// modulo 256; the two particles of a half-wave are paired so that they read
// at the same offsets (see the kappa pairing in the kernel), which the LDS
// serves at its full 16-byte rate.
//
// Weights: every lane evaluates its own node of beta (and beta') by Horner from
// its row of the coefficient table, in powers of t - 1/2 (the centred form
// keeps FP32 cancellation small); the group shares them with DPP
// row_newbcast.  (Folding the broadcast into the FMAs as their DPP operand
// issues fewer instructions but measures slower.)  Sums are FP64 for FP64
// storage and FP32 otherwise.
#include <type_traits>

#include "device_common.h"
#include "launch.h"
#include "ptk_internal.h"

namespace ptk {

enum { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2, ST_F16 = 3 };

// 16-bit storage: the nodes are widened to FP32 (exactly) when they are staged
// into the LDS ring, so the sums read the same 16-byte nodes as FP32 storage
// and spend no instruction on conversions; HBM moves the 6-byte nodes.
template <int ST>
struct StoreT {
  using acc = float;
  static constexpr int T = kTileF32;   // tile edge in cells
  static constexpr int NB = 16;        // LDS bytes per node
  static constexpr int GB = 6;         // global (stored) bytes per node
  static constexpr int THREADS = 512;
};
template <>
struct StoreT<ST_F32> {
  using acc = float;
  static constexpr int T = kTileF32;
  static constexpr int NB = 16;
  static constexpr int GB = 12;
  static constexpr int THREADS = 512;
};
template <>
struct StoreT<ST_F64> {
  using acc = double;
  static constexpr int T = kTileF64;
  static constexpr int NB = 32;
  static constexpr int GB = 24;
  static constexpr int THREADS = 512;
};

template <int ST, int I>
struct Geom {
  static constexpr int T = StoreT<ST>::T;
  static constexpr int TX = T + I - 1;                   // halo tile edge in nodes
  static constexpr int NB = StoreT<ST>::NB;
  static constexpr int RP = TX * NB;                      // row pitch
  // plane pitch, = 128 mod 256: the two half-rows of a particle read planes
  // one ring slot apart.  16-byte nodes: the half-rows cover the two 128-byte
  // halves of the banks.  32-byte (FP64) nodes, read 16 bytes at a time at a
  // 32-byte stride: the halves of a node are swapped in odd slots (lds_put),
  // so the half-rows read the even and the odd 16-byte slots.
  static constexpr int PL = TX * RP + ((128 - (TX * RP) % 256) + 256) % 256;
  static constexpr int R = (kWindow + I - 1 + 1) / 2 * 2;  // ring slots (even): the planes one window touches
  static constexpr int LDS = R * PL;
  // nodes per staged chunk: 48 bytes of FP64 and FP32 nodes, 24 of 16-bit
  // ones (four nodes, as FP32: every thread stages about as many nodes)
  static constexpr int CB = StoreT<ST>::GB == 6 ? 24 : 48;
  static constexpr int G = CB / StoreT<ST>::GB;
  static constexpr int RG = (TX + G - 1) / G;             // chunks per halo row
  static constexpr int UNITS_PER_PLANE = TX * RG;
  static constexpr int THREADS = StoreT<ST>::THREADS;
  static constexpr int PRE = (kWindow * UNITS_PER_PLANE + THREADS - 1) / THREADS;  // chunks per thread
};

// ---- DPP helpers (rows of 16 lanes = one particle group).  Every control
// used here reads a lane of the same row, so no lane keeps an old value and
// the moves need no initialised destination.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
// 64-bit moves: one v_mov_b64_dpp for row_newbcast (the only control DPP
// has for 64-bit operands; the compiler splits the others into two 32-bit
// moves).  A 64-bit broadcast issues as fast as a 32-bit one.
// (the builtin's result is given a 64-bit type explicitly: inside a
// template the front end types the generic builtin's call as int)
template <int CTRL>
__device__ __forceinline__ long dpp64(long v) {
  const long r = __builtin_amdgcn_update_dpp(0L, v, CTRL, 0xF, 0xF, true);
  return r;
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  return __builtin_bit_cast(double, dpp64<CTRL>(__builtin_bit_cast(long, v)));
}
// value of lane L of this row
template <int L, typename V>
__device__ __forceinline__ V bcast(V v) {
  return dpp<0x150 + L>(v);
}
// lanes 0-7 of the row get lane L0's value, lanes 8-15 lane L1's: the second
// move writes only DPP banks 2 and 3 (lanes 8-15) over the first
template <int L0, int L1>
__device__ __forceinline__ float bcast2(float v) {
  const int a = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x150 + L0, 0xF, 0xF, true);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(a, __builtin_bit_cast(int, v), 0x150 + L1, 0xF, 0xC, false));
}
template <int L0, int L1>
__device__ __forceinline__ long bcast2_64(long b) {
  const long a = __builtin_amdgcn_update_dpp(0L, b, 0x150 + L0, 0xF, 0xF, true);
  const long r = __builtin_amdgcn_update_dpp(a, b, 0x150 + L1, 0xF, 0xC, false);
  return r;
}
template <int L0, int L1>
__device__ __forceinline__ double bcast2(double v) {
  return __builtin_bit_cast(double, bcast2_64<L0, L1>(__builtin_bit_cast(long, v)));
}

// sum over the 16 lanes of the row (every lane gets the total)
template <typename V>
__device__ __forceinline__ V rowsum(V v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}

// Reduce-scatter of a particle's three value partials over the 16 lanes of a
// row (lane l16 = j + 8h): after it, lane (h, j) holds the row's total of
// value 2h + (j >> 2) (value 3 is the zero padding), summed over all 16 lanes.
// Five DPP additions instead of three full row sums (twelve).
template <typename V>
__device__ __forceinline__ V rowsum_scatter3(const V* e, int j, int h) {
  const V z = (V)0;
  // lanes l and l^8 (row_ror:8): the h = 0 half keeps values 0, 1, the h = 1
  // half keeps 2 and the padding
  const V k0 = h ? e[2] : e[0], k1 = h ? z : e[1];
  const V s0 = h ? e[0] : e[2], s1 = h ? e[1] : z;
  const V f0 = k0 + dpp<0x128>(s0);
  const V f1 = k1 + dpp<0x128>(s1);
  // lanes j and 7 - j of a half (row_half_mirror): j < 4 keeps f0, j >= 4 f1
  const bool hi = (j & 4) != 0;
  V g = (hi ? f1 : f0) + dpp<0x141>(hi ? f0 : f1);
  g += dpp<0xB1>(g);  // quad_perm [1,0,3,2]
  g += dpp<0x4E>(g);  // quad_perm [2,3,0,1]
  return g;
}

// ---- node access
// copy node q of a 48-byte chunk (12 words) into LDS at byte offset `off`.
// FP64 nodes (32 bytes) in odd ring slots are stored with their halves
// swapped, (z, pad) then (x, y): the two half-rows of a particle read planes
// of opposite slot parity, so reading (x, y) first puts them on opposite
// 16-byte slots of the banks.
template <int ST>
__device__ __forceinline__ void lds_put(unsigned char* smem, int off, const uint32_t* w, int q, bool odd_slot) {
  if constexpr (ST == ST_F32) {
    *(uint4*)(smem + off) = make_uint4(w[3 * q], w[3 * q + 1], w[3 * q + 2], 0u);
  } else if constexpr (ST == ST_F64) {
    const int sxy = odd_slot ? 16 : 0;
    *(uint4*)(smem + off + sxy) = make_uint4(w[6 * q], w[6 * q + 1], w[6 * q + 2], w[6 * q + 3]);
    *(uint4*)(smem + off + 16 - sxy) = make_uint4(w[6 * q + 4], w[6 * q + 5], 0u, 0u);
  } else {
    const int k = 3 * q;
    const uint32_t h0 = (w[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu;
    const uint32_t h1 = (w[(k + 1) >> 1] >> (((k + 1) & 1) * 16)) & 0xFFFFu;
    const uint32_t h2 = (w[(k + 2) >> 1] >> (((k + 2) & 1) * 16)) & 0xFFFFu;
    float f0, f1, f2;
    if constexpr (ST == ST_BF16) {
      f0 = __uint_as_float(h0 << 16);
      f1 = __uint_as_float(h1 << 16);
      f2 = __uint_as_float(h2 << 16);
    } else {
      f0 = __half2float(__ushort_as_half((unsigned short)h0));
      f1 = __half2float(__ushort_as_half((unsigned short)h1));
      f2 = __half2float(__ushort_as_half((unsigned short)h2));
    }
    *(float4*)(smem + off) = make_float4(f0, f1, f2, 0.f);
  }
}

// read a node; the caller consumes the unused fourth word (`keep`) in an empty
// asm statement so the compiler issues one full 16-byte read (ds_read_b128)
// instead of a slower b96.  sxy: byte offset of an FP64 node's (x, y) half
// (16 in odd ring slots, see lds_put).
template <int ST, typename V>
__device__ __forceinline__ void lds_get(const unsigned char* smem, int off, V* v, uint32_t& keep, int sxy) {
  if constexpr (ST == ST_F32) {
    const float4 f = *(const float4*)(smem + off);
    v[0] = f.x;
    v[1] = f.y;
    v[2] = f.z;
    keep = __float_as_uint(f.w);
  } else if constexpr (ST == ST_F64) {
    const double2 a = *(const double2*)(smem + off + sxy);
    const double2 b = *(const double2*)(smem + off + 16 - sxy);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    keep = (uint32_t)__double_as_longlong(b.y);
  } else {
    // 16-bit storage, widened at staging
    const float4 f = *(const float4*)(smem + off);
    v[0] = f.x;
    v[1] = f.y;
    v[2] = f.z;
    keep = __float_as_uint(f.w);
  }
}

// An empty asm that reads a prefetched register, placed where every path
// needs the load complete anyway: then no load into the register is still
// pending on any path when the next prefetch reuses it (the compiler would
// otherwise wait there for every outstanding load, the ones just issued
// included).
__device__ __forceinline__ void settle(uint32_t v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void settle(double v) {
  settle((uint32_t)__double_as_longlong(v));
  settle((uint32_t)((unsigned long long)__double_as_longlong(v) >> 32));
}
__device__ __forceinline__ void settle(const uint4& v) {
  settle(v.x);
  settle(v.y);
  settle(v.z);
  settle(v.w);
}

// f(integral_constant<int, K>) for K = B .. E-1
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Row of I coefficients of the lane's node from the workgroup's LDS copy of
// the table, read when a round needs it instead of being held in registers
// for the whole launch (the registers go to LDS reads in flight).  The row's
// offset passes through an empty asm statement each time, so the compiler
// cannot hoist the reads out of the particle loop; the pointer itself stays
// visibly an LDS pointer (laundering it would turn the reads into flat loads,
// whose waits also wait for every global load in flight).
template <int I, typename V>
__device__ __forceinline__ void coef_row(const V* tab, int off, V* c) {
  asm volatile("" : "+v"(off));
  const V* row = tab + off;
  if constexpr (sizeof(V) == 4) {
#pragma unroll
    for (int p = 0; p < I; p += 4) {
      const float4 f = *(const float4*)(row + p);
      c[p] = f.x;
      if (p + 1 < I) c[p + 1] = f.y;
      if (p + 2 < I) c[p + 2] = f.z;
      if (p + 3 < I) c[p + 3] = f.w;
    }
  } else {
#pragma unroll
    for (int p = 0; p < I; p += 2) {
      const double2 f = *(const double2*)(row + p);
      c[p] = f.x;
      c[p + 1] = f.y;
    }
  }
}

template <int NC, typename V>
__device__ __forceinline__ V horner(const V* c, V t) {
  V acc = c[NC - 1];
#pragma unroll
  for (int p = NC - 2; p >= 0; --p) acc = fma(acc, t, c[p]);
  return acc;
}

// load unit u (one chunk of G nodes of a halo row of plane zp) from HBM.  The
// load is unconditional (a chunk outside the padded field reads the field's
// first chunk instead and is reported invalid), so the compiler keeps it in
// flight rather than waiting for it at a branch merge.
template <int ST, int I>
__device__ __forceinline__ bool load_unit(const InterpArgs& a, int64_t x0, int64_t y0, int64_t zp, int u,
                                          uint4* c) {
  using Gm = Geom<ST, I>;
  const int g = u % Gm::RG;
  const int r = u / Gm::RG;
  const int64_t Y = y0 + r, X = x0 + (int64_t)g * Gm::G;
  const bool ok = zp < a.P && Y < a.P && X < a.P;
  const int64_t off = ok ? zp * a.plane_pitch + Y * a.row_pitch + X * StoreT<ST>::GB : 0;
  const uint4* src = (const uint4*)((const unsigned char*)a.field + off);
  c[0] = src[0];
  if constexpr (Gm::CB == 24) {
    const uint2 t = *(const uint2*)(src + 1);
    c[1] = make_uint4(t.x, t.y, 0u, 0u);
    c[2] = make_uint4(0u, 0u, 0u, 0u);
  } else {
    c[1] = src[1];
    c[2] = src[2];
  }
  return ok;
}

template <int ST, int I>
__device__ __forceinline__ void store_unit(unsigned char* smem, int64_t zp, int u, const uint4* c) {
  using Gm = Geom<ST, I>;
  const int g = u % Gm::RG;
  const int r = u / Gm::RG;
  const uint32_t w[12] = {c[0].x, c[0].y, c[0].z, c[0].w, c[1].x, c[1].y,
                          c[1].z, c[1].w, c[2].x, c[2].y, c[2].z, c[2].w};
  const int slot = (int)((uint32_t)zp % (uint32_t)Gm::R);  // plane indices are below 2^31
#pragma unroll
  for (int q = 0; q < Gm::G; ++q) {
    const int x = g * Gm::G + q;
    if (x < Gm::TX) lds_put<ST>(smem, slot * Gm::PL + r * Gm::RP + x * Gm::NB, w, q, (slot & 1) != 0);
  }
}

// Reference value U(z) of padded plane zp for a tile whose halo starts at
// (x0, y0): the plane's node nearest the tile's centre (clamped into the
// padded field; a plane beyond it is never stored).
__device__ __forceinline__ float3 plane_ref(const InterpArgs& a, int64_t x0, int64_t y0, int64_t zp, int tx) {
  const int64_t X = min(x0 + tx / 2, a.P - 1), Y = min(y0 + tx / 2, a.P - 1), Z = min(zp, a.P - 1);
  const float* p = (const float*)((const unsigned char*)a.field + Z * a.plane_pitch + Y * a.row_pitch + X * 12);
  return make_float3(p[0], p[1], p[2]);
}

// store_unit for FP32 nodes held relative to the plane's reference: every
// component minus U(z) (one FP32 rounding of the difference)
template <int ST, int I>
__device__ __forceinline__ void store_unit_shifted(unsigned char* smem, int64_t zp, int u, const uint4* c, float3 U) {
  static_assert(ST == ST_F32, "plane references are used with FP32 nodes");
  const float uu[3] = {U.x, U.y, U.z};
  uint4 d[3];
  const uint32_t* w = (const uint32_t*)c;
  uint32_t* o = (uint32_t*)d;
#pragma unroll
  for (int e = 0; e < 12; ++e) o[e] = __float_as_uint(__uint_as_float(w[e]) - uu[e % 3]);
  store_unit<ST, I>(smem, zp, u, d);
}

// One particle: 16 lanes (this lane owns x1 offset j and the planes whose ring
// slot has parity h).
// Leaves in r the 3 values (and 9 gradient entries) summed over the group.
template <int ST, int I, bool GRAD, typename V>
__device__ __forceinline__ void particle_sums(const unsigned char* smem, const float4* uref, const V* ctab,
                                              const V* cvreg, int j, int jj, int h, V t1, V t2, V t3, int l1, int l2,
                                              int z3, V* r) {
  using Gm = Geom<ST, I>;
  constexpr int NB = Gm::NB, RP = Gm::RP, PL = Gm::PL, R = Gm::R;
  constexpr int HALF = I / 2;
  // planes of this lane: k = 2m + h, m = 0..I/2-1; the two halves read planes
  // one ring slot apart (or R - 1 apart across the wrap; R is even), an odd
  // number of plane pitches
  // weights: lanes 0-7 evaluate beta_j(t2), lanes 8-15 beta_j(t3); all lanes beta_j(t1)
  const V tsel = h ? t3 : t2;
  // the gradient kernels read their coefficient rows from LDS here (their
  // registers are needed for the sums); the value kernels pass register rows
  V cvl[GRAD ? I : 1];
  if constexpr (GRAD) coef_row<I>(ctab, jj * I, cvl);
  const V* cv = GRAD ? cvl : cvreg;
  const V wsel = horner<I>(cv, tsel);
  V w1 = horner<I>(cv, t1);
  if (j >= I) w1 = (V)0;
  V w2[I], w3[HALF];
  V d1 = (V)0, dw2[I], dw3[HALF];
  {
#define PTK_B2(k) if constexpr ((k) < I) w2[k] = bcast<k>(wsel);
    PTK_B2(0) PTK_B2(1) PTK_B2(2) PTK_B2(3) PTK_B2(4) PTK_B2(5) PTK_B2(6) PTK_B2(7)
#undef PTK_B2
#define PTK_B3(m) if constexpr ((m) < HALF) w3[m] = bcast2<8 + 2 * (m), 9 + 2 * (m)>(wsel);
    PTK_B3(0) PTK_B3(1) PTK_B3(2) PTK_B3(3)
#undef PTK_B3
    if constexpr (GRAD) {
      V cd[I];
      coef_row<I>(ctab, I * I + jj * I, cd);
      const V dsel = horner<I - 1>(cd, tsel);
      d1 = horner<I - 1>(cd, t1);
      if (j >= I) d1 = (V)0;
#define PTK_D2(k) if constexpr ((k) < I) dw2[k] = bcast<k>(dsel);
      PTK_D2(0) PTK_D2(1) PTK_D2(2) PTK_D2(3) PTK_D2(4) PTK_D2(5) PTK_D2(6) PTK_D2(7)
#undef PTK_D2
#define PTK_D3(m) if constexpr ((m) < HALF) dw3[m] = bcast2<8 + 2 * (m), 9 + 2 * (m)>(dsel);
      PTK_D3(0) PTK_D3(1) PTK_D3(2) PTK_D3(3)
#undef PTK_D3
    }
  }
  // contraction: x2 over all rows per plane, x3 over this lane's planes
  const int noff = l2 * RP + (l1 + jj) * NB;
  const int s0 = (z3 + h) % R;
  // every plane of this lane has the slot parity of s0 (R is even)
  const int sxy = (s0 & 1) * 16;
  V acc[3] = {0, 0, 0}, ad2[3] = {0, 0, 0}, ad3[3] = {0, 0, 0};
  // the unused fourth word of every 16-byte node read is folded into `sink`
  // by an empty (schedulable) asm, so the reads stay 16 bytes wide without a
  // wait after each one; one asm at the end keeps the chain alive
  uint32_t sink = 0;
  // FP32 gradients: the ring holds every plane z relative to a reference
  // value U(z) of that plane (see plane_ref); the x2 sums of a plane then get
  // U(z) - U(z_c) added back, z_c the particle's own plane, and the value
  // U(z_c) at the end.  Exact arithmetic is unchanged (the weights sum to 1,
  // their derivatives to 0, along every axis), while the FP32 roundings of the
  // large sums scale with the variation of u within a plane of the tile
  // instead of with u.
  constexpr bool SHIFT = GRAD && ST == ST_F32;
  float4 uc = make_float4(0.f, 0.f, 0.f, 0.f);
  if constexpr (SHIFT) uc = uref[(z3 + I / 2 - 1) % R];
#pragma unroll
  for (int m = 0; m < HALF; ++m) {
    const int slot = s0 + 2 * m < R ? s0 + 2 * m : s0 + 2 * m - R;
    const int base = slot * PL + noff;
    V s[3] = {0, 0, 0}, sd[3] = {0, 0, 0};
    if constexpr (SHIFT) {
      // the plane's U(z) - U(z_c) starts the x2 sum (the x2 derivative sum
      // needs none: the derivative weights sum to 0)
      const float4 um = uref[slot];
      s[0] = um.x - uc.x;
      s[1] = um.y - uc.y;
      s[2] = um.z - uc.z;
    }
    // rows read together before use: four for values, two for gradients
    // (four would pass the 128-VGPR budget of two workgroups per CU and spill)
    constexpr int G = GRAD ? 2 : (I % 4 == 0 ? 4 : 2);
#pragma unroll
    for (int g = 0; g < I; g += G) {
      V v[G][3];
      uint32_t keep[G];
#pragma unroll
      for (int k = 0; k < G; ++k) lds_get<ST>(smem, base + (g + k) * RP, v[k], keep[k], sxy);
#pragma unroll
      for (int k = 0; k < G; ++k) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          s[q] = fma(w2[g + k], v[k][q], s[q]);
          if constexpr (GRAD) sd[q] = fma(dw2[g + k], v[k][q], sd[q]);
        }
        asm("" : "+v"(sink) : "v"(keep[k]));
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      acc[q] = fma(w3[m], s[q], acc[q]);
      if constexpr (GRAD) {
        ad3[q] = fma(dw3[m], s[q], ad3[q]);
        ad2[q] = fma(w3[m], sd[q], ad2[q]);
      }
    }
  }
  asm volatile("" ::"v"(sink));
  // x1 weight, then the sum over the group's 16 lanes.  Values: r[q] = u_q,
  // r[3 + 3q + b] = d u_q / d x_b (before the 1/delta factor).
  V e[GRAD ? 12 : 3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    e[q] = w1 * acc[q];
    if constexpr (GRAD) {
      e[3 + 3 * q + 0] = d1 * acc[q];
      e[3 + 3 * q + 1] = w1 * ad2[q];
      e[3 + 3 * q + 2] = w1 * ad3[q];
    }
  }
  if constexpr (!GRAD) {
    // lane (h, j) gets the total of value 2h + (j >> 2)
    r[0] = rowsum_scatter3(e, j, h);
  } else {
    // reduce-scatter: lanes l and l^8 split the 12 values 6/6, then lanes j and
    // 7-j of each half split their 6 values 3/3, then each quad sums its 3.
    // Lane l16 ends with the totals of values 6*(l16/8) + 3*((l16/4)&1) + k,
    // k = 0..2, in r[k].
    const int b2 = (j >> 2) & 1;
    V f[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const V keep = h ? e[6 + k] : e[k];
      const V send = h ? e[k] : e[6 + k];
      f[k] = keep + dpp<0x128>(send);  // row_ror:8, the lane 8 away
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const V keep = b2 ? f[3 + k] : f[k];
      const V send = b2 ? f[k] : f[3 + k];
      V g = keep + dpp<0x141>(send);   // row_half_mirror, lane 7-j
      g += dpp<0xB1>(g);
      g += dpp<0x4E>(g);
      r[k] = g;
    }
    // lanes 0-3 hold the values: add back the particle plane's reference
    if constexpr (SHIFT) {
      if (h == 0 && b2 == 0) {
        r[0] += uc.x;
        r[1] += uc.y;
        r[2] += uc.z;
      }
    }
  }
}

// SPARSE: for launches with few particles per window -- visit only the
// non-empty windows of each segment and fill the ring afresh for each,
// instead of sweeping every plane.  Two workgroups per CU for FP32 and 16-bit
// storage; FP64 nodes fill the LDS of one.
template <int ST, int I, bool GRAD, bool SPARSE>
// the second bound is waves per SIMD: two 512-thread workgroups per CU are 4
// (at most 128 VGPRs), one is 2
__global__ __launch_bounds__(StoreT<ST>::THREADS, ST == ST_F64 ? 2 : 4) void k_interp(InterpArgs a) {
  using V = typename StoreT<ST>::acc;
  using Gm = Geom<ST, I>;
  constexpr int T = Gm::T;
  constexpr int W = kWindow;
  constexpr int NT = Gm::THREADS;
  constexpr int GL = 16;                 // lanes per particle
  constexpr int GROUPS = NT / GL;        // particles per round
  constexpr int NV = GRAD ? 12 : 3;
  constexpr int CH = NT / 3 / GROUPS * GROUPS;  // particles located per chunk: one thread per coordinate
  // particle record: t1, t2, t3 (V) at 0; cells l1, l2, z3 (u16) at 32;
  // destination indices (u32) of the values at 40 and of the gradient at 44
  constexpr int RECB = 48;
  __shared__ __attribute__((aligned(16))) unsigned char smem[Gm::LDS];
  __shared__ __attribute__((aligned(16))) unsigned char recs[CH * RECB];
  // Particle pairing: a half-wave holds two particles, and a 16-byte read
  // runs at full rate only when both quarter-waves read at the same offset
  // modulo 256 bytes.  A particle's reads sit at offsets (up to a constant
  // common to all lanes) 16 * kappa mod 256: kappa = 8 (c3 mod 2) + TX l2 + l1
  // mod 16 for 16-byte nodes (plane pitch = 128 mod 256, row pitch = 16 TX),
  // 9 (c3 mod 2) + 2 TX l2 + 2 l1 for 32-byte FP64 nodes (row pitch 32 TX;
  // the (x, y) half of a node in an odd slot sits 16 bytes in).  The rounds
  // take the window's particles in an order that puts equal kappa side by
  // side: rord[] lists record indices, pairs of each kappa first, then the
  // unpaired ones.  Each particle's arithmetic is unchanged.
  constexpr bool PAIR = GL == 16 && (Gm::NB == 16 || Gm::NB == 32);
  __shared__ uint8_t rord[PAIR ? CH : 1];
  __shared__ __attribute__((aligned(16))) int kcnt[16];
  static_assert(CH <= 255, "record indices fit a byte");
  // FP32 gradient kernels hold the ring's planes relative to a reference
  // value per plane: U(z) of the plane in ring slot s (see particle_sums)
  constexpr bool PSHIFT = GRAD && ST == ST_F32;
  __shared__ float4 uref[PSHIFT ? Gm::R : 1];
  // the references of the planes the next window adds, posted before the
  // barrier that precedes their store
  __shared__ float4 unext[PSHIFT ? W : 1];
  // the bin offsets of this segment's windows, [w_begin, w_end]: read once, so
  // no window waits on a global load to find its range
  __shared__ uint32_t woff[kMaxWps + 1];

  // ---- block -> (tile column, x3 segment); consecutive blocks go round-robin
  // to the 8 XCDs, so XCD x is given a contiguous range of an ordering of the
  // columns by 8 x 8 blocks of columns: the columns an XCD sweeps at the same
  // time are neighbours in x1 and x2, and the halo planes they share are read
  // from its L2
  const int64_t nblk = a.n_tiles * a.nseg;
  const int64_t per_xcd = (nblk + 7) / 8;
  const int64_t b = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (b >= nblk) return;
  const int64_t ord = b / a.nseg;  // position of the column in the blocked order
  const int seg = (int)(b % a.nseg);
  int64_t tile;
  {
    // 32-bit arithmetic: columns per axis and their count are small
    constexpr uint32_t S = 8;
    const uint32_t ntx = (uint32_t)a.ntx, o = (uint32_t)ord;
    const uint32_t band = o / (S * ntx);                // band of S rows of columns
    const uint32_t rows = min(S, ntx - band * S);
    const uint32_t off = o - band * S * ntx;
    const uint32_t sc = off / (rows * S);               // S-wide block within the band
    const uint32_t cols = min(S, ntx - sc * S);
    const uint32_t inner = off - sc * rows * S;
    tile = (int64_t)((band * S + inner / cols) * ntx + sc * S + inner % cols);
  }
  const int64_t w_begin = (int64_t)seg * a.wps;
  const int64_t w_end = min(a.nw, w_begin + a.wps);
  if (w_begin >= w_end) return;
  {
    const int64_t bin0 = tile * a.nw + w_begin;
    for (int e = threadIdx.x; e <= (int)(w_end - w_begin); e += Gm::THREADS) woff[e] = a.offsets[bin0 + e];
    if (threadIdx.x < 16) kcnt[threadIdx.x] = 0;
  }
  const int tx = (int)(tile % a.ntx), ty = (int)(tile / a.ntx);
  const int64_t x0 = (int64_t)tx * T, y0 = (int64_t)ty * T;
  const int tid = threadIdx.x;

  // ---- per-lane constants
  const int l16 = tid & 15;
  const int j = l16 & 7;              // x1 node offset
  const int h = l16 >> 3;             // plane half
  const int jj = j < I ? j : I - 1;
  const int grp = tid / GL;
  // the kernel's coefficient rows (in powers of t - 1/2) in LDS: [2][I][I]
  // values then derivatives; written here, read after the first barrier
  __shared__ __attribute__((aligned(16))) V ctab[2 * I * I];
  {
    const KernelTables* tab = (const KernelTables*)a.coef;
    for (int e = tid; e < 2 * I * I; e += Gm::THREADS) {
      const int d = e / (I * I), rr = (e / I) % I, p = e % I;
      if constexpr (sizeof(V) == 8)
        ctab[e] = d ? tab->cder64[rr][p] : tab->cval64[rr][p];
      else
        ctab[e] = d ? tab->cder32[rr][p] : tab->cval32[rr][p];
    }
  }
  const V* cvrow = ctab + jj * I;
  // value kernels hold their row in registers for the whole launch (a read
  // per round would sit at the head of every round's dependency chain); the
  // gradient kernels, which need their registers for the sums, read both
  // rows from LDS at the start of each round
  V cvr[GRAD ? 1 : I];
  __syncthreads();  // ctab and woff are complete
  if constexpr (!GRAD) {
#pragma unroll
    for (int p = 0; p < I; ++p) cvr[p] = cvrow[p];
  }
  const int N = a.N;
  const double invd = a.invd;

  // ---- fill the ring with the planes window w touches: [W*w, W*w + W + I - 1)
  auto fill = [&](int64_t w) {
    const int64_t z_lo = W * w;
    constexpr int UNITS = (W + I - 1) * Gm::UNITS_PER_PLANE;
    for (int u = tid; u < UNITS; u += NT) {
      uint4 c[3];
      const int pl = u / Gm::UNITS_PER_PLANE, uu = u % Gm::UNITS_PER_PLANE;
      if constexpr (PSHIFT) {
        const float3 U = plane_ref(a, x0, y0, z_lo + pl, Gm::TX);
        if (load_unit<ST, I>(a, x0, y0, z_lo + pl, uu, c)) {
          store_unit_shifted<ST, I>(smem, z_lo + pl, uu, c, U);
          if (uu == 0) uref[(z_lo + pl) % Gm::R] = make_float4(U.x, U.y, U.z, 0.f);
        }
      } else {
        if (load_unit<ST, I>(a, x0, y0, z_lo + pl, uu, c)) store_unit<ST, I>(smem, z_lo + pl, uu, c);
      }
    }
  };

  // ---- software pipeline over windows: while window w is computed, the
  // positions of window w+1, the particle rows of window w+2 and the planes
  // window w+DEPTH adds are in flight (issued in that order, so each wait only
  // covers older loads).  The planes of window v are loaded into buffer
  // v mod DEPTH, DEPTH windows ahead (one for the gradient kernels, which
  // need the registers).  Finding a window's rows (through the bin
  // permutation where positions are read through it) one window before
  // loading their coordinates keeps a window with few particles from waiting
  // on two loads in a row.
  constexpr int DEPTH = (GRAD || ST == ST_BF16 || ST == ST_F16) ? 1 : 2;
  uint4 pre[DEPTH][Gm::PRE][3];
  bool pok[DEPTH][Gm::PRE];
  // window w+1: its particle range, this thread's coordinate and destination
  double pos_x = 0.0;
  uint32_t pos_q = 0u, pos_s = 0u, pos_e = 0u;
  int pos_n = 0;
  // window w+2: its particle range, this thread's row of X and destination
  uint32_t idx_i = 0u, idx_q = 0u, idx_s = 0u, idx_e = 0u;
  int idx_n = 0;
  // the end of window w+3's range, read a window before it is needed
  uint32_t end3 = 0u;

  // (the unit index of a thread is recomputed per window from a laundered
  // thread index: hoisted out of the sweep, these per-thread addresses would
  // hold registers through the particle rounds)
  auto utid = [&]() {
    int t = tid;
    asm volatile("" : "+v"(t));
    return t;
  };
  auto issue_planes = [&](int64_t wn, uint4 (&pre)[Gm::PRE][3], bool (&ok)[Gm::PRE]) {
    const int64_t zn = W * wn + I - 1;  // planes window wn adds: [zn, zn + W)
    const int t0 = utid();
#pragma unroll
    for (int k = 0; k < Gm::PRE; ++k) {
      const int uraw = t0 + k * NT;
      const int u = min(uraw, W * Gm::UNITS_PER_PLANE - 1);
      const int pl = u / Gm::UNITS_PER_PLANE, uu = u % Gm::UNITS_PER_PLANE;
      ok[k] = load_unit<ST, I>(a, x0, y0, zn + pl, uu, pre[k]) && uraw < W * Gm::UNITS_PER_PLANE && wn < w_end;
    }
  };
  // FP32 gradient kernels: the reference node of every plane (plane_ref's
  // node, clamped into the padded field) lies in one unit of the plane, the
  // same unit index for every plane of the column; the thread that holds it
  // in its prefetch registers posts its value before the barrier that
  // precedes store_planes, so no thread waits on a global load to shift its
  // nodes.
  int ref_unit = 0, ref_q = 0;
  if constexpr (PSHIFT) {
    const int rx = (int)min((int64_t)(Gm::TX / 2), a.P - 1 - x0), ry = (int)min((int64_t)(Gm::TX / 2), a.P - 1 - y0);
    ref_unit = ry * Gm::RG + rx / Gm::G;
    ref_q = rx % Gm::G;
  }
  auto post_refs = [&](const uint4 (&pre)[Gm::PRE][3], const bool (&ok)[Gm::PRE]) {
    if constexpr (PSHIFT) {
      const int t0 = utid();
#pragma unroll
      for (int k = 0; k < Gm::PRE; ++k) {
        const int u = t0 + k * NT;
        if (ok[k] && u % Gm::UNITS_PER_PLANE == ref_unit) {
          // node ref_q of the chunk, picked by selects (a run-time index into
          // the registers would move them to scratch memory)
          const uint32_t wd[12] = {pre[k][0].x, pre[k][0].y, pre[k][0].z, pre[k][0].w, pre[k][1].x, pre[k][1].y,
                                   pre[k][1].z, pre[k][1].w, pre[k][2].x, pre[k][2].y, pre[k][2].z, pre[k][2].w};
          uint32_t n0 = wd[0], n1 = wd[1], n2 = wd[2];
#pragma unroll
          for (int q = 1; q < Gm::G; ++q) {
            n0 = ref_q == q ? wd[3 * q] : n0;
            n1 = ref_q == q ? wd[3 * q + 1] : n1;
            n2 = ref_q == q ? wd[3 * q + 2] : n2;
          }
          unext[u / Gm::UNITS_PER_PLANE] = make_float4(__uint_as_float(n0), __uint_as_float(n1), __uint_as_float(n2), 0.f);
        }
      }
    }
  };
  auto store_planes = [&](int64_t wn, const uint4 (&pre)[Gm::PRE][3], const bool (&ok)[Gm::PRE]) {
    const int64_t zn = W * wn + I - 1;
#pragma unroll
    for (int k = 0; k < Gm::PRE; ++k)
      for (int c = 0; c < 3; ++c) settle(pre[k][c]);
    const int t0 = utid();
#pragma unroll
    for (int k = 0; k < Gm::PRE; ++k) {
      const int u = t0 + k * NT;
      if (ok[k]) {
        const int pl = u / Gm::UNITS_PER_PLANE, uu = u % Gm::UNITS_PER_PLANE;
        if constexpr (PSHIFT) {
          const float4 U4 = unext[pl];
          const float3 U = make_float3(U4.x, U4.y, U4.z);
          store_unit_shifted<ST, I>(smem, zn + pl, uu, pre[k], U);
          if (uu == 0) uref[(uint32_t)(zn + pl) % (uint32_t)Gm::R] = U4;
        } else {
          store_unit<ST, I>(smem, zn + pl, uu, pre[k]);
        }
      }
    }
  };
  // position coordinate + destination index of particle c0 + tid/3 (clamped, unconditional)
  auto issue_pos = [&](uint32_t c0, int n, double& xv, uint32_t& qv) {
    const int pi = min(tid / 3, max(n - 1, 0));
    const int64_t p = min((int64_t)c0 + pi, (int64_t)a.np - 1);
    const int64_t xi = a.xrow ? (int64_t)a.xrow[p] : p;
    xv = a.X[3 * xi + tid % 3];
    // axis-1 threads fetch the gradient destination, the others the value one
    const uint32_t* src = (tid % 3 == 1 && a.grad_orig) ? a.grad_orig : a.orig;
    qv = src ? src[p] : (uint32_t)p;
  };
  // steps 1-3 of Sec. 2.2 once per coordinate: one thread per (particle, axis)
  // steps 1-3 of Sec. 2.2 once per coordinate: one thread per (particle, axis)
  auto write_rec = [&](int64_t wr, int n, double xv, uint32_t qv) {
    settle(xv);
    settle(qv);
    if (tid < 3 * n) {
      const int pi = tid / 3, ax = tid % 3;
      int c;
      double td;
      locate(xv, N, invd, &c, &td);
      // the cell must lie in the bin's tile column and window (binning and
      // kernel locate alike); a particle outside them is reported, and its
      // record clamped so that every LDS read stays inside the ring
      int lc;
      bool inside;
      if (ax == 0) {
        lc = c - (int)x0;
        inside = lc >= 0 && lc < T;
        lc = min(max(lc, 0), T - 1);
      } else if (ax == 1) {
        lc = c - (int)y0;
        inside = lc >= 0 && lc < T;
        lc = min(max(lc, 0), T - 1);
      } else {
        inside = (int64_t)c >= W * wr && (int64_t)c < W * wr + W;
        lc = (int)min(max((int64_t)c, W * wr), W * wr + W - 1);
      }
      if (!inside) atomicOr(a.flag, kFlagBinning);
      // the weights are polynomials in t - 1/2 (exact in binary64 for t >= 1/4
      // by Sterbenz's lemma and for every t that is a multiple of 2^-53;
      // below that it rounds by less than 2^-54)
      unsigned char* rp = recs + pi * RECB;
      if constexpr (sizeof(V) == 8)
        ((double*)rp)[ax] = td - 0.5;
      else
        ((float*)rp)[ax] = (float)(td - 0.5);
      ((uint16_t*)(rp + 32))[ax] = (uint16_t)lc;
      if (ax == 0) *(uint32_t*)(rp + 40) = qv;
      if (ax == 1) *(uint32_t*)(rp + 44) = qv;
    }
  };
  // The round order of a chunk whose records are complete (after a barrier):
  // rank_kappa ranks each particle within its kappa bucket (thread = particle,
  // one LDS atomic); after a second barrier, place puts the pairs of every
  // bucket first, bucket by bucket, then one left-over particle of each bucket
  // with an odd count.  Returns / takes kappa + 16 * rank.
  auto rank_kappa = [&](int n) -> int {
    int kr = 0;
    if constexpr (PAIR) {
      if (tid < n) {
        const uint2 lc = *(const uint2*)(recs + tid * RECB + 32);
        const int l1 = (int)(lc.x & 0xFFFFu), l2 = (int)(lc.x >> 16), c3 = (int)(lc.y & 0xFFFFu);
        // 16-byte nodes: offsets 16 (8 p + TX l2 + l1); 32-byte nodes, whose
        // (x, y) half sits 16 bytes in where the slot parity p is odd:
        // 16 (9 p + 2 TX l2 + 2 l1), modulo 256 (p = c3 mod 2)
        const int kap = Gm::NB == 16 ? (8 * (c3 & 1) + Gm::TX * l2 + l1) & 15
                                     : (9 * (c3 & 1) + 2 * Gm::TX * l2 + 2 * l1) & 15;
        kr = kap + 16 * atomicAdd(&kcnt[kap], 1);
      }
    }
    return kr;
  };
  auto place = [&](int n, int kr) {
    if constexpr (PAIR) {
      if ((tid & ~63) < n) {  // waves holding a particle of the chunk
        // per 16-lane row: bucket l16's (pairs, odd) packed in one word, and
        // its exclusive prefix over the buckets (DPP scan within the row)
        const int cnt = kcnt[l16];
        const int v = (cnt >> 1) | ((cnt & 1) << 16);
        int inc = v;
        inc += __builtin_amdgcn_mov_dpp(inc, 0x111, 0xF, 0xF, true);  // row_shr:1
        inc += __builtin_amdgcn_mov_dpp(inc, 0x112, 0xF, 0xF, true);  // row_shr:2
        inc += __builtin_amdgcn_mov_dpp(inc, 0x114, 0xF, 0xF, true);  // row_shr:4
        inc += __builtin_amdgcn_mov_dpp(inc, 0x118, 0xF, 0xF, true);  // row_shr:8
        const int total = __builtin_amdgcn_readlane(inc, 15);
        const int kap = kr & 15, rank = kr >> 4;
        const int row0 = (tid & 63) & ~15;
        const int before = __shfl(inc - v, row0 + kap);
        const int own = __shfl(v, row0 + kap);
        if (tid < n) {
          const int pos = rank < 2 * (own & 0xFFFF) ? 2 * (before & 0xFFFF) + rank
                                                     : 2 * (total & 0xFFFF) + (before >> 16);
          rord[pos] = (uint8_t)tid;
        }
      }
    }
  };
  auto compute_chunk = [&](int n) __attribute__((always_inline)) {
    const int wave_grp0 = __builtin_amdgcn_readfirstlane(grp & ~(64 / GL - 1));  // first group of this wave
    // the pairing's counters are free again (every placement read them before
    // the barrier that started this chunk; the next count follows a barrier)
    if (PAIR && tid < 16) kcnt[tid] = 0;
    for (int r0 = 0; r0 < n; r0 += GROUPS) {
      if (r0 + wave_grp0 >= n) break;  // nothing left for this wave: its SIMD serves other waves
      const int pi = r0 + grp;
      const bool active = pi < n;
      const int ri = PAIR ? (int)rord[active ? pi : n - 1] : (active ? pi : n - 1);
      const unsigned char* rp = recs + ri * RECB;
      V t1, t2, t3;
      if constexpr (sizeof(V) == 8) {
        const double2 ta = *(const double2*)rp;
        const double2 tb = *(const double2*)(rp + 16);
        t1 = ta.x;
        t2 = ta.y;
        t3 = tb.x;
      } else {
        const float4 tf = *(const float4*)rp;
        t1 = tf.x;
        t2 = tf.y;
        t3 = tf.z;
        // the unused word rides on t3 (arriving together), so the read stays
        // 16 bytes wide and the next one is issued before either is waited on
        asm("" : "+v"(t3) : "v"(tf.w));
      }
      const uint4 lc = *(const uint4*)(rp + 32);
      const int l1 = (int)(lc.x & 0xFFFFu), l2 = (int)(lc.x >> 16), z3 = (int)(lc.y & 0xFFFFu);
      V r[3];
      particle_sums<ST, I, GRAD>(smem, uref, ctab, cvr, j, jj, h, t1, t2, t3, l1, l2, z3, r);
      // which of its totals this lane writes, and which value that is: the
      // gradient kernels hold three (value 6h + 3((j >> 2) & 1) + k in r[k],
      // lane j & 3 writes k = j & 3); the value kernels one (value 2h +
      // (j >> 2) in r[0], written by lane j & 3 = 0)
      const int sub = GRAD ? (l16 & 3)
                           : ((j & 3) == 0 && 2 * h + (j >> 2) < 3) ? 0 : 3;
      const int ev = GRAD ? 6 * (l16 >> 3) + 3 * ((l16 >> 2) & 1) + (l16 & 3) : 2 * h + (j >> 2);
      V val = r[0];
      val = sub == 1 ? r[1] : val;
      val = sub == 2 ? r[2] : val;
      if (active && sub < 3) {
        const int64_t q = (int64_t)(ev < 3 ? lc.z : lc.w);
        if (ev < 3) {
          if (ST == ST_BF16 || ST == ST_F16)
            val *= (V)(ev == 0 ? a.scale[0] : ev == 1 ? a.scale[1] : a.scale[2]);
          if (a.out) {
            if (a.out_f64)
              ((double*)a.out)[3 * q + ev] = (double)val;
            else
              ((float*)a.out)[3 * q + ev] = (float)val;
          }
        } else {
          val *= (V)invd;
          if (ST == ST_BF16 || ST == ST_F16)
            val *= (V)(ev < 6 ? a.scale[0] : ev < 9 ? a.scale[1] : a.scale[2]);
          if (a.out_f64)
            ((double*)a.grad)[9 * q + (ev - 3)] = (double)val;
          else
            ((float*)a.grad)[9 * q + (ev - 3)] = (float)val;
        }
      }
    }
  };
  // the range [start, end) of a window and this thread's X row and
  // destination index in it
  auto issue_window_idx = [&](uint32_t start, uint32_t end, uint32_t& iv, uint32_t& qv, int& nv, uint32_t& s_out,
                              uint32_t& e_out) {
    s_out = start;
    e_out = end;
    nv = (int)min((int64_t)CH, (int64_t)end - (int64_t)start);
    // unconditional (clamped to a particle of the launch: the segment has
    // one), so every path has the same loads in flight and no wait for them
    // lands early
    const int pi = min(tid / 3, max(nv - 1, 0));
    const int64_t p = min((int64_t)start + pi, (int64_t)a.np - 1);
    iv = a.xrow ? a.xrow[p] : (uint32_t)p;
    // axis-1 threads fetch the gradient destination, the others the value one
    const uint32_t* src = (tid % 3 == 1 && a.grad_orig) ? a.grad_orig : a.orig;
    qv = src ? src[p] : (uint32_t)p;
  };
  // the coordinate of that row (iv is always a row of X)
  auto issue_window_x = [&](uint32_t iv, double& xv) { xv = a.X[3 * (int64_t)iv + tid % 3]; };
  // one window: records of w are in LDS, the ring holds w's planes, the
  // position registers hold w's range; plane buffer B (w - w_begin mod DEPTH)
  // receives the planes of w+DEPTH
  auto window = [&](int64_t w, auto B_) {
    constexpr int B = decltype(B_)::value;
    constexpr int B1 = (B + 1) % DEPTH;
    const uint32_t start = pos_s, end = pos_e;
    // positions of w+1 from the rows found a window ago, then the rows of w+2
    // (the rows' loads are waited for before any new load is issued)
    settle(idx_i);
    settle(idx_q);
    pos_s = idx_s;
    pos_e = idx_e;
    pos_n = idx_n;
    pos_q = idx_q;
    issue_window_x(idx_i, pos_x);
    issue_window_idx(idx_e, w + 2 < w_end ? end3 : idx_e, idx_i, idx_q, idx_n, idx_s, idx_e);
    if (w + 3 < w_end) end3 = woff[w + 4 - w_begin];
    issue_planes(w + DEPTH, pre[B], pok[B]);
    __syncthreads();  // records of w and the ring are complete
    int n = (int)min((int64_t)CH, (int64_t)end - (int64_t)start);
    compute_chunk(n);
    // rare: more than CH particles in the window; later chunks are loaded in place
    for (uint32_t c0 = start + CH; c0 < end; c0 += CH) {
      const int m = (int)min((int64_t)CH, (int64_t)end - (int64_t)c0);
      double xm;
      uint32_t qm;
      issue_pos(c0, m, xm, qm);
      __syncthreads();
      write_rec(w, m, xm, qm);
      __syncthreads();
      if constexpr (PAIR) {
        const int kr = rank_kappa(m);
        __syncthreads();
        place(m, kr);
        __syncthreads();
      }
      compute_chunk(m);
    }
    post_refs(pre[B1], pok[B1]);
    __syncthreads();  // every read of this window's ring slots and records is done
    // the ring holds at least the planes one window touches: w+1's new planes
    // replace planes no later window reads; then w+1's records
    store_planes(w + 1, pre[B1], pok[B1]);
    if (w + 1 < w_end) {
      write_rec(w + 1, pos_n, pos_x, pos_q);
      if constexpr (PAIR) {
        __syncthreads();  // w+1's records are complete
        const int kr = rank_kappa(pos_n);
        __syncthreads();  // every count is in
        place(pos_n, kr);
      }
    }
  };

  {
    if (woff[0] == woff[w_end - w_begin]) return;  // no particle in this segment
    if constexpr (SPARSE) {
      for (int64_t w = w_begin; w < w_end; ++w) {
        const uint32_t start = woff[w - w_begin], end = woff[w + 1 - w_begin];
        if (start == end) continue;
        fill(w);
        for (uint32_t c0 = start; c0 < end; c0 += CH) {
          const int m = (int)min((int64_t)CH, (int64_t)end - (int64_t)c0);
          double xm;
          uint32_t qm;
          issue_pos(c0, m, xm, qm);
          write_rec(w, m, xm, qm);
          __syncthreads();  // ring and records complete
          if constexpr (PAIR) {
            const int kr = rank_kappa(m);
            __syncthreads();
            place(m, kr);
            __syncthreads();
          }
          compute_chunk(m);
          __syncthreads();  // every read done before the next fill
        }
      }
      return;
    }
  }
  fill(w_begin);
  __syncthreads();

  // ---- prologue: records of the first window, the rows of the second and
  // planes of w_begin+1 .. w_begin+DEPTH-1 in flight
  {
    double xv = 0.0;
    uint32_t qv = 0, iv = 0;
    int nv = 0;
    issue_window_idx(woff[0], woff[1], iv, qv, nv, pos_s, pos_e);
    issue_window_x(iv, xv);
    write_rec(w_begin, nv, xv, qv);
    if constexpr (PAIR) {
      __syncthreads();
      const int kr = rank_kappa(nv);
      __syncthreads();
      place(nv, kr);
    }
    issue_window_idx(pos_e, w_begin + 1 < w_end ? woff[2] : pos_e, idx_i, idx_q, idx_n, idx_s, idx_e);
    if (w_begin + 2 < w_end) end3 = woff[3];
  }
  static_for<1, DEPTH>([&](auto K) { issue_planes(w_begin + decltype(K)::value, pre[decltype(K)::value], pok[decltype(K)::value]); });
  // windows in pairs so that every plane buffer index is a constant (single
  // windows when there is one buffer)
  static_assert(DEPTH == 1 || DEPTH == 2, "window pairs cover plane depths 1 and 2");
  if constexpr (DEPTH == 2) {
    for (int64_t w = w_begin; w < w_end; w += 2) {
      window(w, std::integral_constant<int, 0>{});
      if (w + 1 < w_end) {
        window(w + 1, std::integral_constant<int, 1>{});
      } else {
        // (the loads of the buffer the skipped window would have stored are
        // settled on this path too; see settle)
#pragma unroll
        for (int k = 0; k < Gm::PRE; ++k)
          for (int c = 0; c < 3; ++c) settle(pre[0][k][c]);
      }
    }
  } else {
    for (int64_t w = w_begin; w < w_end; ++w) window(w, std::integral_constant<int, 0>{});
  }
}

template <int ST, int I>
static hipError_t launch_one(const InterpArgs& a, hipStream_t s) {
  const int64_t nblk = a.n_tiles * a.nseg;
  const int64_t grid = (nblk + 7) / 8 * 8;
  if (grid == 0) return hipSuccess;
  constexpr int NT = StoreT<ST>::THREADS;
  // sparse when one fresh ring per particle loads fewer planes than the sweep
  const bool sparse = a.np * (kWindow + I - 1) < a.n_tiles * a.nw * kWindow;
  if (a.grad) {
    if (sparse)
      k_interp<ST, I, true, true><<<(unsigned)grid, NT, 0, s>>>(a);
    else
      k_interp<ST, I, true, false><<<(unsigned)grid, NT, 0, s>>>(a);
  } else {
    if (sparse)
      k_interp<ST, I, false, true><<<(unsigned)grid, NT, 0, s>>>(a);
    else
      k_interp<ST, I, false, false><<<(unsigned)grid, NT, 0, s>>>(a);
  }
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
