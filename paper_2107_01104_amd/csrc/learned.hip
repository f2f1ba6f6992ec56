// Learned correction form: stencil features and the I = 4 Lagrange sum at
// particles, and a 195-128-128-3 SiLU network whose two hidden-layer products
// run on the matrix cores (BF16 operands, FP32 sums) -- training (forward,
// backward, Adam) and inference on binned particles.
//
// Matrix-core tiles: v_mfma_f32_32x32x16_bf16.  Lane l holds, of a 32 x 16 A
// tile, row l%32 and the 8 consecutive k starting at 8*(l/32); of a 16 x 32 B
// tile, column l%32 and the same k; of the 32 x 32 FP32 result, column l%32
// and rows 8*(v/4) + 4*(l/32) + v%4 in register v.  A workgroup of 4 waves
// takes 64 rows (particles or training pairs); wave w owns hidden units
// [32w, 32w+32) in the forward products.
#include "device_common.h"
#include "launch.h"
#include "ptk_internal.h"

namespace ptk {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int NF = kLearnedNFeat;   // 195 features
constexpr int FP = kLearnedPitch;   // 200: global feature row pitch
constexpr int K1 = 208;             // layer-1 k extent, padded to 13 x 16
constexpr int NH = 128, NO = 3;
constexpr int oW1 = 0, oB1 = NH * NF, oW2 = oB1 + NH, oB2 = oW2 + NH * NH, oW3 = oB2 + NH, oB3 = oW3 + NO * NH;
static_assert(oB3 + NO == kLearnedNParams, "parameter layout");
constexpr int ROWS = 64, NT = 256;
// LDS pitches in BF16 elements: rows of 16 x odd bytes, so that 32 lanes
// reading 16 bytes each from 32 consecutive rows cover all banks
constexpr int PX = 216;   // features (K1 + 8)
constexpr int PH = 136;   // hidden activations
constexpr int PT = 72;    // transposed tiles: 64 rows + 8
constexpr int PH2 = 132;  // FP32 h2 rows

__device__ __forceinline__ bf16x8 frag(const uint16_t* base, int pitch, int row, int k) {
  return __builtin_bit_cast(bf16x8, *(const uint4*)(base + row * pitch + k));
}
__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// logistic function through the hardware exponential and reciprocal
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}
// row of result register v of this lane within a 32-row tile
__device__ __forceinline__ int acc_row(int v, int hi) { return 8 * (v >> 2) + 4 * hi + (v & 3); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// two FP32 values rounded to BF16 (nearest even, one conversion instruction)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const bf16x2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// value of lane L of this lane's group of 4
template <int L>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, L * 0x55, 0xF, 0xF, true);
}

__device__ __forceinline__ float quad_sum(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
  v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, true));
  return v;
}

typedef float f32x4a __attribute__((ext_vector_type(4), aligned(4)));

// Steps 1-3 of Sec. 2.2 for the particle of this lane's group of 4: lane k
// (k < 3) locates coordinate k, and the group shares cells and offsets.
// Returns whether this lane's coordinate is inside the domain (lane 3: true).
__device__ __forceinline__ bool locate_quad_x(double x, int k3, int N, double invd, int* c, double* td) {
  const bool ok = k3 == 3 || in_domain(x);
  int cc;
  double tt;
  locate(ok ? x : 0.0, N, invd, &cc, &tt);
  const long long tb = __double_as_longlong(tt);
  int lo = (int)(tb & 0xFFFFFFFFll), hi = (int)(tb >> 32);
#define PTK_Q(d)                                                                                   \
  c[d] = quad_bcast<d>(cc);                                                                        \
  td[d] = __longlong_as_double(((long long)(unsigned)quad_bcast<d>(hi) << 32) | (unsigned)quad_bcast<d>(lo));
  PTK_Q(0) PTK_Q(1) PTK_Q(2)
#undef PTK_Q
  return ok;
}

// the same from the particle's row of X: thread k3 loads coordinate min(k3, 2)
__device__ __forceinline__ bool locate_quad(const double* Xp, int k3, int N, double invd, int* c, double* td) {
  return locate_quad_x(Xp[k3 < 3 ? k3 : 2], k3, N, invd, c, td);
}

// One quarter of a particle's 4 x 4 x 4 stencil (the x3 plane k3): the loads
// of its 4 rows (4 nodes each: 12 consecutive floats, 4-byte aligned), ...
__device__ __forceinline__ void stencil_issue(const LearnedField& f, const int* c, int k3, float4 (&q)[4][3]) {
  const int64_t z = c[2] - 1 + k3 + f.halo_lo;
  const unsigned char* plane = (const unsigned char*)f.field + z * f.plane_pitch;
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    const int64_t y = c[1] - 1 + k2 + f.halo_lo;
    const f32x4a* row = (const f32x4a*)((const float*)(plane + y * f.row_pitch) + 3 * (c[0] - 1 + f.halo_lo));
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const f32x4a r = row[e];
      q[k2][e] = make_float4(r.x, r.y, r.z, r.w);
    }
  }
}

// ... and from them its 48 BF16 features, packed in pairs into fe[24] in
// feature order, and its part of the Lagrange I = 4 sum
__device__ __forceinline__ void stencil_sums(const LearnedField& f, const double* td, int k3, const float4 (&q)[4][3],
                                             uint32_t* fe, float* u) {
  float w[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float t = (float)td[d];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float acc = f.l4[j][3];
#pragma unroll
      for (int p = 2; p >= 0; --p) acc = fmaf(acc, t, f.l4[j][p]);
      w[d][j] = acc;
    }
  }
  u[0] = u[1] = u[2] = 0.f;
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    const float4 q0 = q[k2][0], q1 = q[k2][1], q2 = q[k2][2];
    const float v[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
    const float w23 = w[2][k3] * w[1][k2];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      const float ww = w23 * w[0][k1];
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = fmaf(ww, v[3 * k1 + a], u[a]);
    }
#pragma unroll
    for (int qq = 0; qq < 6; ++qq) fe[6 * k2 + qq] = pack_bf16(v[2 * qq], v[2 * qq + 1]);
  }
}

__device__ __forceinline__ void stencil_plane(const LearnedField& f, const int* c, const double* td, int k3,
                                              uint32_t* fe, float* u) {
  float4 q[4][3];
  stencil_issue(f, c, k3, q);
  stencil_sums(f, td, k3, q, fe, u);
}

// ---------------------------------------------------------------- pairs
// thread = (particle, x3 plane of its stencil); caller order
__global__ __launch_bounds__(NT) void k_pairs(LearnedField f, const double* X, int64_t n, const float* uwide,
                                              uint16_t* feat, float* target, int* flag) {
  const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t p = min(g >> 2, n - 1);
  const int k3 = (int)(g & 3);
  const bool active = (g >> 2) < n;
  int c[3];
  double td[3];
  const bool ok = locate_quad(X + 3 * p, k3, f.N, f.invd, c, td);
  if (active && !ok) atomicOr(flag, kFlagDomain);
  uint32_t fe[24];
  float u[3];
  stencil_plane(f, c, td, k3, fe, u);
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = quad_sum(u[a]);
  if (!active) return;
  if (feat) {
    uint2* dst = (uint2*)(feat + p * FP + 48 * k3);
#pragma unroll
    for (int q = 0; q < 12; ++q) dst[q] = make_uint2(fe[2 * q], fe[2 * q + 1]);
    if (k3 == 0) {
      uint32_t* tail = (uint32_t*)(feat + p * FP + 192);
      tail[0] = pack_bf16((float)td[0], (float)td[1]);
      tail[1] = (uint32_t)to_bf16((float)td[2]);
      tail[2] = 0u;
      tail[3] = 0u;
    }
  }
  if (target && k3 == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) target[3 * p + a] = uwide[3 * p + a] - u[a];
  }
}

// ---------------------------------------------------------------- forward
// Hidden layer 1 for the 64 rows whose features are in sX: h1 (BF16) in sH1
// (and its transpose in sH1t if given), the pre-activations' derivatives
// (training) in ds1.  Ends with the barrier after which h1 is complete and sX
// is dead.
template <bool TRAIN>
__device__ __forceinline__ void hidden_layer1(const uint16_t* sX, uint16_t* sH1, uint16_t* sH1t,
                                              const bf16x8 (&bw1)[13], float bias1, f32x16 (&ds1)[2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r32 = lane & 31, hi = lane >> 5;
  const int J = 32 * wave + r32;
  f32x16 acc[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[rt][v] = 0.f;
  // the A fragments of step s + 1 are read while step s's products run; in
  // inference an empty asm with a memory clobber ends every step, so the
  // compiler reads no further ahead (holding all 26 fragments would take 104
  // registers that inference spends on the next chunk's stencil loads)
  bf16x8 an[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) an[rt] = frag(sX, PX, 32 * rt + r32, 8 * hi);
#pragma unroll
  for (int s = 0; s < 13; ++s) {
    const bf16x8 a0 = an[0], a1 = an[1];
    if (s + 1 < 13) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) an[rt] = frag(sX, PX, 32 * rt + r32, 16 * (s + 1) + 8 * hi);
    }
    acc[0] = mfma(a0, bw1[s], acc[0]);
    acc[1] = mfma(a1, bw1[s], acc[1]);
    if constexpr (!TRAIN) asm volatile("" ::: "memory");
  }
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int v0 = 0; v0 < 16; v0 += 4) {
      float h[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float z = acc[rt][v0 + q] + bias1;
        h[q] = silu(z);
        if constexpr (TRAIN) ds1[rt][v0 + q] = dsilu(z);
      }
      const uint32_t p01 = pack_bf16(h[0], h[1]), p23 = pack_bf16(h[2], h[3]);
      const int r0 = 32 * rt + acc_row(v0, hi);
      sH1[r0 * PH + J] = (uint16_t)p01;
      sH1[(r0 + 1) * PH + J] = (uint16_t)(p01 >> 16);
      sH1[(r0 + 2) * PH + J] = (uint16_t)p23;
      sH1[(r0 + 3) * PH + J] = (uint16_t)(p23 >> 16);
      if (sH1t) *(uint2*)(sH1t + J * PT + r0) = make_uint2(p01, p23);
    }
  __syncthreads();  // h1 complete; sX is dead from here on
}

// Training's forward pass: layer 1 as above, then h2 (FP32) in sH2 and its
// pre-activations' derivatives in ds2 (the backward pass reads h2 by rows).
// sX and sH2 may alias.
__device__ __forceinline__ void forward_hidden(const uint16_t* sX, uint16_t* sH1, uint16_t* sH1t, float* sH2,
                                               const bf16x8 (&bw1)[13], const bf16x8 (&bw2)[8], float bias1,
                                               float bias2, f32x16 (&ds1)[2], f32x16 (&ds2)[2]) {
  hidden_layer1<true>(sX, sH1, sH1t, bw1, bias1, ds1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r32 = lane & 31, hi = lane >> 5;
  const int J = 32 * wave + r32;
  f32x16 acc[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[rt][v] = 0.f;
  bf16x8 an[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) an[rt] = frag(sH1, PH, 32 * rt + r32, 8 * hi);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const bf16x8 a0 = an[0], a1 = an[1];
    if (s + 1 < 8) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) an[rt] = frag(sH1, PH, 32 * rt + r32, 16 * (s + 1) + 8 * hi);
    }
    acc[0] = mfma(a0, bw2[s], acc[0]);
    acc[1] = mfma(a1, bw2[s], acc[1]);
  }
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float z = acc[rt][v] + bias2;
      sH2[(32 * rt + acc_row(v, hi)) * PH2 + J] = silu(z);
      ds2[rt][v] = dsilu(z);
    }
  __syncthreads();  // h2 complete
}

// Inference: hidden layer 2 with the operands swapped (W2 rows as the A tile,
// h1 rows as the B tile), so that lane l holds particle 32 rt + l % 32 and,
// in register v, the wave's hidden unit 32 wave + acc_row(v, l / 32); then
// the output layer straight from those registers.  Each lane adds its 16
// units' h2 W3 products, the wave's two lane halves add theirs (lane l ^ 32
// holds the other 16 units of the same particles), and lanes l < 32 leave the
// wave's sums in sY[wave][row][a].  Ends with the barrier after which sY is
// complete.  Training keeps the FP32 h2 tile (forward_hidden): its backward
// pass reads h2 by rows.
__device__ __forceinline__ void infer_layer2_out(const uint16_t* sH1, const bf16x8 (&bw2)[8], const float* sB2,
                                                 const float* sW3, float* sY) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r32 = lane & 31, hi = lane >> 5;
  f32x16 acc[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[rt][v] = 0.f;
  bf16x8 bn[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) bn[rt] = frag(sH1, PH, 32 * rt + r32, 8 * hi);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const bf16x8 b0 = bn[0], b1 = bn[1];
    if (s + 1 < 8) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) bn[rt] = frag(sH1, PH, 32 * rt + r32, 16 * (s + 1) + 8 * hi);
    }
    acc[0] = mfma(bw2[s], b0, acc[0]);
    acc[1] = mfma(bw2[s], b1, acc[1]);
    asm volatile("" ::: "memory");
  }
  float y[2][NO];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int a = 0; a < NO; ++a) y[rt][a] = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // registers 4k .. 4k+3 hold units u0 .. u0+3
    const int u0 = 32 * wave + 8 * k + 4 * hi;
    const float4 b = *(const float4*)(sB2 + u0);
    const float4 w0 = *(const float4*)(sW3 + u0), w1 = *(const float4*)(sW3 + NH + u0),
                 w2 = *(const float4*)(sW3 + 2 * NH + u0);
    const float bb[4] = {b.x, b.y, b.z, b.w};
    const float ww[NO][4] = {{w0.x, w0.y, w0.z, w0.w}, {w1.x, w1.y, w1.z, w1.w}, {w2.x, w2.y, w2.z, w2.w}};
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float h = silu(acc[rt][4 * k + q] + bb[q]);
#pragma unroll
        for (int a = 0; a < NO; ++a) y[rt][a] = fmaf(h, ww[a][q], y[rt][a]);
      }
  }
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int a = 0; a < NO; ++a) y[rt][a] += __shfl_xor(y[rt][a], 32);
  if (hi == 0) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int a = 0; a < NO; ++a) sY[(wave * ROWS + 32 * rt + r32) * NO + a] = y[rt][a];
  }
  __syncthreads();  // every wave's sums are in sY
}

// y[r][a] = b3[a] + sum_c h2[r][c] W3[a][c] for thread t < 192 (r = t/3, a = t%3)
__device__ __forceinline__ float output_layer(const float* sH2, const float* sW3, const float* b3, int t) {
  const int r = t / 3, a = t - 3 * (t / 3);
  const float4* h = (const float4*)(sH2 + r * PH2);
  const float4* w = (const float4*)(sW3 + a * NH);
  float y0 = 0.f, y1 = 0.f;
#pragma unroll 8
  for (int c = 0; c < NH / 4; c += 2) {
    const float4 h0 = h[c], w0 = w[c], h1 = h[c + 1], w1 = w[c + 1];
    y0 = fmaf(h0.x, w0.x, y0);
    y0 = fmaf(h0.y, w0.y, y0);
    y0 = fmaf(h0.z, w0.z, y0);
    y0 = fmaf(h0.w, w0.w, y0);
    y1 = fmaf(h1.x, w1.x, y1);
    y1 = fmaf(h1.y, w1.y, y1);
    y1 = fmaf(h1.z, w1.z, y1);
    y1 = fmaf(h1.w, w1.w, y1);
  }
  return b3[a] + (y0 + y1);
}

__device__ __forceinline__ void load_weight_frags(const uint16_t* w1b, const uint16_t* w2b, bf16x8 (&bw1)[13],
                                                  bf16x8 (&bw2)[8]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int J = 32 * wave + (lane & 31), hi = lane >> 5;
#pragma unroll
  for (int s = 0; s < 13; ++s) bw1[s] = frag(w1b, K1, J, 16 * s + 8 * hi);
#pragma unroll
  for (int s = 0; s < 8; ++s) bw2[s] = frag(w2b, NH, J, 16 * s + 8 * hi);
}

// ---------------------------------------------------------------- training
// One workgroup: 64 consecutive pairs starting at row0 = 64 * blockIdx.x.
// Writes its part of the gradient (parameter layout) to gpart[blockIdx.x] and
// its sum of squared errors to lpart[blockIdx.x].
__global__ __launch_bounds__(NT, 1) void k_forward_backward(const uint16_t* feat, const float* target, int64_t batch,
                                                            const float* params, const uint16_t* w1b,
                                                            const uint16_t* w2b, const uint16_t* w2bt, float* gpart,
                                                            float* lpart, const uint16_t* feat_next) {
  // LDS regions (bytes): R0 transposed features [224][PT]; R1 transposed h1
  // [128][PT]; R2 features [64][PX] -> h2 FP32 [64][PH2] -> dz2 [64][PH] +
  // transposed dz2 [128][PT]; R3 h1 [64][PH] -> transposed dz1 [128][PT]
  constexpr int R0 = 224 * PT * 2, R1 = NH * PT * 2;
  constexpr int R2 = ROWS * PH * 2 + NH * PT * 2;  // the largest of its three uses
  static_assert(R2 >= ROWS * PX * 2 && R2 >= ROWS * PH2 * 4, "R2 size");
  constexpr int R3 = NH * PT * 2;
  static_assert(R3 >= ROWS * PH * 2, "R3 size");
  __shared__ __attribute__((aligned(16))) unsigned char lds[R0 + R1 + R2 + R3];
  __shared__ float sW3[NO * NH];
  __shared__ float sdy[ROWS * NO];
  __shared__ float sdw3[2 * NO * NH];  // dW3 sums of the two halves of the rows
  __shared__ float sred[NT / 64];
  uint16_t* sXt = (uint16_t*)lds;
  uint16_t* sH1t = (uint16_t*)(lds + R0);
  unsigned char* r2 = lds + R0 + R1;
  uint16_t* sX = (uint16_t*)r2;
  float* sH2 = (float*)r2;
  uint16_t* sdZ2 = (uint16_t*)r2;
  uint16_t* sdZ2t = (uint16_t*)(r2 + ROWS * PH * 2);
  uint16_t* sH1 = (uint16_t*)(lds + R0 + R1 + R2);
  uint16_t* sdZ1t = sH1;

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6, r32 = lane & 31, hi = lane >> 5;
  const int J = 32 * wave + r32;
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  float* gp = gpart + (int64_t)blockIdx.x * kLearnedNParams;

  // features -> sX (row-major) and sXt (transposed); entries 195.. are zero.
  // This thread's 16-byte pieces are loaded together (unconditionally, from
  // a clamped address), then stored.
  constexpr int FE = ROWS * (K1 / 8), FI = (FE + NT - 1) / NT;
  uint4 fq[FI];
#pragma unroll
  for (int i = 0; i < FI; ++i) {
    const int e = min(t + i * NT, FE - 1);
    const int r = e / (K1 / 8), k0 = (e % (K1 / 8)) * 8;
    fq[i] = *(const uint4*)(feat + (row0 + r) * FP + (k0 < FP ? k0 : 0));
  }
  // the same rows of the next step's batch, read now so that they are in
  // this XCD's L2 when that step's workgroup (same block index, same XCD)
  // starts; their registers are consumed only at the end of the kernel
  uint4 fnext[FI];
  if (feat_next) {
#pragma unroll
    for (int i = 0; i < FI; ++i) {
      const int e = min(t + i * NT, FE - 1);
      const int r = e / (K1 / 8), k0 = (e % (K1 / 8)) * 8;
      fnext[i] = *(const uint4*)(feat_next + (row0 + r) * FP + (k0 < FP ? k0 : 0));
    }
  }
#pragma unroll
  for (int i = 0; i < FI; ++i) {
    const int e = t + i * NT;
    if (e >= FE) break;
    const int r = e / (K1 / 8), k0 = (e % (K1 / 8)) * 8;
    uint16_t v[8];
    {
      const uint32_t w[4] = {fq[i].x, fq[i].y, fq[i].z, fq[i].w};
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = k0 < FP ? (uint16_t)(w[j >> 1] >> (16 * (j & 1))) : (uint16_t)0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k0 + j >= NF) v[j] = 0;
    *(uint4*)(sX + r * PX + k0) = make_uint4((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                                             (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16));
  }
  __syncthreads();  // sX complete
  // sXt from sX: item (k, 8 rows from r0) per thread, consecutive threads on
  // consecutive k, so the 2-byte reads of a row are contiguous and the
  // 16-byte writes (row pitch 144 bytes) fall on distinct banks within each
  // quarter-wave; rows k >= K1 are zero
  for (int i = t; i < 224 * (ROWS / 8); i += NT) {
    const int k = i % 224, r0 = (i / 224) * 8;
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = k < K1 ? sX[(r0 + j) * PX + k] : (uint16_t)0;
    *(uint4*)(sXt + k * PT + r0) = make_uint4((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                                              (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16));
  }
  for (int e = t; e < NO * NH; e += NT) sW3[e] = params[oW3 + e];
  bf16x8 bw1[13], bw2[8];
  load_weight_frags(w1b, w2b, bw1, bw2);
  const float bias1 = params[oB1 + J], bias2 = params[oB2 + J];
  __syncthreads();

  f32x16 ds1[2], ds2[2];
  forward_hidden(sX, sH1, sH1t, sH2, bw1, bw2, bias1, bias2, ds1, ds2);

  // output layer, loss and dy = 2 (y - target) / (3 batch)
  float se = 0.f;
  if (t < ROWS * NO) {
    const float y = output_layer(sH2, sW3, params + oB3, t);
    const float d = y - target[(row0 + t / 3) * NO + t % 3];
    se = d * d;
    sdy[t] = 2.0f * d / (float)(NO * batch);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) se += __shfl_xor(se, o);
  if (lane == 0) sred[wave] = se;
  __syncthreads();
  if (t == 0) lpart[blockIdx.x] = (sred[0] + sred[1]) + (sred[2] + sred[3]);
  // dW3[a][c] = sum_r dy[r][a] h2[r][c]: thread (c, half) sums its half of
  // the rows for the three a (the halves are added after the barrier);
  // db3[a] = sum_r dy[r][a]
  static_assert(NT == 2 * NH, "dW3 split");
  {
    const int c = t & (NH - 1), r0 = (t / NH) * (ROWS / 2);
    float g[NO] = {0.f, 0.f, 0.f};
#pragma unroll 8
    for (int r = r0; r < r0 + ROWS / 2; ++r) {
      const float h = sH2[r * PH2 + c];
#pragma unroll
      for (int a = 0; a < NO; ++a) g[a] = fmaf(sdy[r * NO + a], h, g[a]);
    }
#pragma unroll
    for (int a = 0; a < NO; ++a) sdw3[(t / NH) * NO * NH + a * NH + c] = g[a];
  }
  if (t < NO) {
    float g = 0.f;
    for (int r = 0; r < ROWS; ++r) g += sdy[r * NO + t];
    gp[oB3 + t] = g;
  }
  __syncthreads();  // every read of h2 is done: R2 now takes dz2
  for (int o = t; o < NO * NH; o += NT) gp[oW3 + o] = sdw3[o] + sdw3[NO * NH + o];

  // dz2 = (dy W3) * silu'(z2), stored as BF16 row-major and transposed
  {
    float db = 0.f;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v0 = 0; v0 < 16; v0 += 4) {
        float dz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 32 * rt + acc_row(v0 + q, hi);
          const float dh = sdy[r * NO] * sW3[J] + sdy[r * NO + 1] * sW3[NH + J] + sdy[r * NO + 2] * sW3[2 * NH + J];
          dz[q] = dh * ds2[rt][v0 + q];
          db += dz[q];
        }
        const uint32_t p01 = pack_bf16(dz[0], dz[1]), p23 = pack_bf16(dz[2], dz[3]);
        const int r0 = 32 * rt + acc_row(v0, hi);
        sdZ2[r0 * PH + J] = (uint16_t)p01;
        sdZ2[(r0 + 1) * PH + J] = (uint16_t)(p01 >> 16);
        sdZ2[(r0 + 2) * PH + J] = (uint16_t)p23;
        sdZ2[(r0 + 3) * PH + J] = (uint16_t)(p23 >> 16);
        *(uint2*)(sdZ2t + J * PT + r0) = make_uint2(p01, p23);
      }
    db += __shfl_xor(db, 32);
    if (hi == 0) gp[oB2 + J] = db;
  }
  __syncthreads();

  // dh1 = dz2 W2 (unit J of layer 1), dz1 = dh1 * silu'(z1) -> transposed BF16
  {
    f32x16 acc[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[rt][v] = 0.f;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const bf16x8 b = frag(w2bt, NH, J, 16 * s + 8 * hi);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) acc[rt] = mfma(frag(sdZ2, PH, 32 * rt + r32, 16 * s + 8 * hi), b, acc[rt]);
    }
    float db = 0.f;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v0 = 0; v0 < 16; v0 += 4) {
        float dz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          dz[q] = acc[rt][v0 + q] * ds1[rt][v0 + q];
          db += dz[q];
        }
        *(uint2*)(sdZ1t + J * PT + 32 * rt + acc_row(v0, hi)) =
            make_uint2(pack_bf16(dz[0], dz[1]), pack_bf16(dz[2], dz[3]));
      }
    db += __shfl_xor(db, 32);
    if (hi == 0) gp[oB1 + J] = db;
  }
  // dW2[i][j] = sum_r dz2[r][i] h1[r][j]: rows i of tile `wave`, 4 column tiles
  {
    f32x16 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[nt][v] = 0.f;
#pragma unroll
    for (int s = 0; s < ROWS / 16; ++s) {
      const bf16x8 a = frag(sdZ2t, PT, 32 * wave + r32, 16 * s + 8 * hi);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(a, frag(sH1t, PT, 32 * nt + r32, 16 * s + 8 * hi), acc[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 16; ++v) gp[oW2 + (32 * wave + acc_row(v, hi)) * NH + 32 * nt + r32] = acc[nt][v];
  }
  __syncthreads();  // dz1 complete
  // dW1[i][f] = sum_r dz1[r][i] x[r][f] for f < 195: 7 column tiles in two passes
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    constexpr int NTP = 4;
    f32x16 acc[NTP];
#pragma unroll
    for (int q = 0; q < NTP; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[q][v] = 0.f;
    const int nt0 = pass * NTP;
    const int ntn = pass == 0 ? NTP : 7 - NTP;
#pragma unroll
    for (int s = 0; s < ROWS / 16; ++s) {
      const bf16x8 a = frag(sdZ1t, PT, 32 * wave + r32, 16 * s + 8 * hi);
#pragma unroll
      for (int q = 0; q < NTP; ++q)
        if (q < ntn) acc[q] = mfma(a, frag(sXt, PT, 32 * (nt0 + q) + r32, 16 * s + 8 * hi), acc[q]);
    }
#pragma unroll
    for (int q = 0; q < NTP; ++q) {
      const int fcol = 32 * (nt0 + q) + r32;
      if (q < ntn && fcol < NF)
#pragma unroll
        for (int v = 0; v < 16; ++v) gp[oW1 + (32 * wave + acc_row(v, hi)) * NF + fcol] = acc[q][v];
    }
  }
  if (feat_next) {
#pragma unroll
    for (int i = 0; i < FI; ++i) asm volatile("" ::"v"(fnext[i].x));
  }
}

// Sum of the workgroups' gradients, then (mode 1) one Adam step with BF16
// copies of W1, W2 (and W2 transposed), (mode 0) the gradient and loss only,
// (mode 2) the BF16 copies only.  A workgroup takes 64 parameters: wave q
// sums the q-th quarter of the partials (consecutive, in order, their loads
// in flight together), and wave 0 adds the four sums in order, so the order
// of every addition is fixed.
constexpr int UPD_E = 64;  // parameters per workgroup of k_update
__global__ __launch_bounds__(NT) void k_update(float* params, float* m, float* v, const float* gpart,
                                               const float* lpart, LearnedUpdate u, uint16_t* w1b, uint16_t* w2b,
                                               uint16_t* w2bt) {
  __shared__ float sq[4][UPD_E];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * UPD_E + lane;
  if (blockIdx.x == 0 && threadIdx.x == 0 && u.loss_out && u.mode != 2) {
    float l = 0.f;
    for (int w = 0; w < u.nparts; ++w) l += lpart[w];
    u.loss_out[0] = l * u.loss_scale;
  }
  float g = 0.f;
  if (u.mode != 2) {
    const int per = (u.nparts + 3) / 4;
    const int w0 = wave * per, w1 = min(u.nparts, w0 + per);
    if (e < kLearnedNParams) {
      int w = w0;
      for (; w + 16 <= w1; w += 16) {
        float part[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) part[k] = gpart[(int64_t)(w + k) * kLearnedNParams + e];
#pragma unroll
        for (int k = 0; k < 16; ++k) g += part[k];
      }
      for (; w < w1; ++w) g += gpart[(int64_t)w * kLearnedNParams + e];
    }
    sq[wave][lane] = g;
    __syncthreads();
    g = ((sq[0][lane] + sq[1][lane]) + sq[2][lane]) + sq[3][lane];
  }
  if (wave != 0 || e >= kLearnedNParams) return;
  float p = params[e];
  if (u.mode != 2) {
    if (u.mode == 0) {
      u.grad_out[e] = g;
      return;
    }
    const float mm = u.beta1 * m[e] + (1.0f - u.beta1) * g;
    const float vv = u.beta2 * v[e] + (1.0f - u.beta2) * g * g;
    m[e] = mm;
    v[e] = vv;
    p -= u.lr * (mm * u.c1) / (sqrtf(vv * u.c2) + u.eps);
    params[e] = p;
  }
  const uint16_t b = to_bf16(p);
  if (e < oB1) {
    w1b[(e / NF) * K1 + e % NF] = b;
  } else if (e >= oW2 && e < oB2) {
    const int j = (e - oW2) / NH, k = (e - oW2) % NH;
    w2b[j * NH + k] = b;
    w2bt[k * NH + j] = b;
  }
}

// ---------------------------------------------------------------- inference
// Particles in bin order (the k-th is the caller's orig[k]; orig is required),
// 64 per chunk;
// every workgroup keeps its layer weights in registers and walks a range of
// chunks.  The loads run a chunk ahead of their use along the chain row
// index -> coordinate -> stencil: while chunk ch's two layers run, chunk
// ch + 1's stencil rows, chunk ch + 2's coordinates and chunk ch + 3's row
// indices are in flight.
__global__ __launch_bounds__(NT, 2) void k_infer(LearnedField f, const double* X, int64_t n, const uint32_t* orig,
                                                 const float* params, const uint16_t* w1b, const uint16_t* w2b,
                                                 float* out, int* flag) {
  constexpr int RX = ROWS * PX * 2;  // features
  __shared__ __attribute__((aligned(16))) unsigned char lds[RX + ROWS * PH * 2];
  __shared__ __attribute__((aligned(16))) float sW3[NO * NH];
  __shared__ __attribute__((aligned(16))) float sB2[NH];
  __shared__ float sY[4 * ROWS * NO];  // the 4 waves' output-layer sums
  __shared__ float sU[ROWS * NO];
  __shared__ float sB3[NO];
  uint16_t* sX = (uint16_t*)lds;
  uint16_t* sH1 = (uint16_t*)(lds + RX);
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int J = 32 * wave + (lane & 31);
  for (int e = t; e < NO * NH; e += NT) sW3[e] = params[oW3 + e];
  if (t < NH) sB2[t] = params[oB2 + t];
  if (t < NO) sB3[t] = params[oB3 + t];
  bf16x8 bw1[13], bw2[8];
  load_weight_frags(w1b, w2b, bw1, bw2);
  const float bias1 = params[oB1 + J];
  f32x16 unused1[2];
  // each block walks a contiguous range of chunks (neighbouring bins, so its
  // stencil reads stay in L2 and in the translation caches); consecutive
  // blocks go round-robin to the 8 XCDs, so XCD x is given a contiguous range
  const int64_t nchunks = (n + ROWS - 1) / ROWS;
  const int64_t per_xcd = gridDim.x / 8;
  const int64_t bid = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const int64_t per_block = (nchunks + gridDim.x - 1) / gridDim.x;
  const int64_t ch_end = min(nchunks, (bid + 1) * per_block);
  const int64_t ch0 = bid * per_block;
  const int kx = (t & 3) < 3 ? (t & 3) : 2;  // the coordinate this thread loads
  // row of X of this thread's particle in chunk ch
  // caller row of bin-ordered particle p (clamped to the last particle;
  // unconditional, so no branch merge waits for the load)
  auto xrow_of = [&](int64_t p) -> uint32_t { return orig[min(p, n - 1)]; };
  auto xrow = [&](int64_t ch) -> uint32_t { return xrow_of(ch * ROWS + (t >> 2)); };
  // At the top of chunk ch: its stencil rows q (with their offsets td and
  // domain check ok), loaded during chunk ch - 1, and chunk ch + 1's
  // coordinate x_n.  Each load's result is consumed before the register is
  // loaded again, and every wait finds the loads it needs issued before the
  // ones still in flight (the counter retires loads in order).
  const int pi = t >> 2, k3 = t & 3;
  float4 q[4][3];
  double td[3];
  bool ok = true;
  double x_n = 0.0;
  if (ch0 < ch_end) {
    const double x_c = X[3 * (int64_t)xrow(ch0) + kx];
    const uint32_t oi = xrow(min(ch0 + 1, ch_end - 1));
    int c[3];
    ok = locate_quad_x(x_c, k3, f.N, f.invd, c, td);
    stencil_issue(f, c, k3, q);
    x_n = X[3 * (int64_t)oi + kx];
  }
  // output thread t < 192 writes component t % 3 of the chunk's particle t / 3
  const int orow = min(t / 3, ROWS - 1), oa = t % 3;
  for (int64_t ch = ch0; ch < ch_end; ++ch) {
    // the caller's row of this thread's output, and chunk ch + 2's rows of X
    const uint32_t o_dst = xrow_of(ch * ROWS + orow);
    const uint32_t oi_nn = xrow(min(ch + 2, ch_end - 1));
    const bool active = ch * ROWS + pi < n;
    if (active && !ok) atomicOr(flag, kFlagDomain);
    uint32_t fe[24];
    float u[3];
    stencil_sums(f, td, k3, q, fe, u);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = quad_sum(u[a]);
    uint16_t* row = sX + pi * PX;
#pragma unroll
    for (int e = 0; e < 12; ++e) *(uint2*)(row + 48 * k3 + 4 * e) = make_uint2(fe[2 * e], fe[2 * e + 1]);
    if (k3 == 0) {
      *(uint32_t*)(row + 192) = pack_bf16((float)td[0], (float)td[1]);
      row[194] = to_bf16((float)td[2]);
      sU[pi * NO] = u[0];
      sU[pi * NO + 1] = u[1];
      sU[pi * NO + 2] = u[2];
    } else if (k3 == 1) {
#pragma unroll
      for (int k = NF; k < PX; ++k) row[k] = 0;
    }
    // the next chunk: locate its particles and put its stencil loads in
    // flight (clamped to the last chunk: the loads are unconditional, so no
    // path waits for them early); then the coordinates of the chunk after it.
    // The empty asm keeps these loads below the use of this chunk's rows, so
    // the two sets of rows are never held at once.
    asm volatile("" ::: "memory");
    {
      int c[3];
      ok = locate_quad_x(x_n, k3, f.N, f.invd, c, td);
      stencil_issue(f, c, k3, q);
      x_n = X[3 * (int64_t)oi_nn + kx];
    }
    __syncthreads();
    hidden_layer1<false>(sX, sH1, nullptr, bw1, bias1, unused1);
    infer_layer2_out(sH1, bw2, sB2, sW3, sY);
    if (t < ROWS * NO) {
      const float* yw = sY + orow * NO + oa;
      const float y = sB3[oa] + ((yw[0] + yw[ROWS * NO]) + (yw[2 * ROWS * NO] + yw[3 * ROWS * NO]));
      if (ch * ROWS + orow < n) out[3 * (int64_t)o_dst + oa] = sU[orow * NO + oa] + y;
    }
    __syncthreads();  // sY and sU are read before the next chunk overwrites them
  }
}

// ---------------------------------------------------------------- audit
__global__ void k_stride_gather(const double* X, int64_t stride, int64_t na, double* Xa) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= na) return;
  const int64_t p = i * stride;
  Xa[3 * i] = X[3 * p];
  Xa[3 * i + 1] = X[3 * p + 1];
  Xa[3 * i + 2] = X[3 * p + 2];
}

// sums[0] = sum |out[k i] - uw[i]|^2, sums[1] = sum |uw[i]|^2 in FP64; one block
__global__ __launch_bounds__(1024) void k_audit(const float* out, int64_t stride, int64_t na, const float* uw,
                                                double* sums) {
  __shared__ double se[1024], sr[1024];
  double e = 0.0, r = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += 1024)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double w = uw[3 * i + a];
      const double d = (double)out[3 * (i * stride) + a] - w;
      e += d * d;
      r += w * w;
    }
  se[threadIdx.x] = e;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      se[threadIdx.x] += se[threadIdx.x + h];
      sr[threadIdx.x] += sr[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[0] = se[0];
    sums[1] = sr[0];
  }
}

}  // namespace

hipError_t launch_learned_pairs(const LearnedField& f, const double* X, int64_t n, const float* uwide,
                                uint16_t* feat, float* target, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (4 * n + NT - 1) / NT;
  k_pairs<<<(unsigned)blocks, NT, 0, s>>>(f, X, n, uwide, feat, target, flag);
  return hipGetLastError();
}

hipError_t launch_learned_forward_backward(const uint16_t* feat, const float* target, int64_t batch,
                                           const float* params, const uint16_t* w1b, const uint16_t* w2b,
                                           const uint16_t* w2bt, float* gpart, float* lpart, hipStream_t s,
                                           const uint16_t* feat_next) {
  if (batch <= 0 || batch % ROWS) return hipErrorInvalidValue;
  k_forward_backward<<<(unsigned)(batch / ROWS), NT, 0, s>>>(feat, target, batch, params, w1b, w2b, w2bt, gpart,
                                                             lpart, feat_next);
  return hipGetLastError();
}

hipError_t launch_learned_update(float* params, float* m, float* v, const float* gpart, const float* lpart,
                                 const LearnedUpdate& u, uint16_t* w1b, uint16_t* w2b, uint16_t* w2bt,
                                 hipStream_t s) {
  const int blocks = (kLearnedNParams + UPD_E - 1) / UPD_E;
  k_update<<<blocks, NT, 0, s>>>(params, m, v, gpart, lpart, u, w1b, w2b, w2bt);
  return hipGetLastError();
}

hipError_t launch_learned_infer(const LearnedField& f, const double* X, int64_t n, const uint32_t* orig,
                                const float* params, const uint16_t* w1b, const uint16_t* w2b, float* out,
                                int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (!orig) return hipErrorInvalidValue;  // the kernel reads every particle's row through it
  const int64_t nchunks = (n + ROWS - 1) / ROWS;
  const int64_t grid = min((nchunks + 7) / 8 * 8, (int64_t)256 * 2 * 4);  // a multiple of the 8 XCDs
  k_infer<<<(unsigned)grid, NT, 0, s>>>(f, X, n, orig, params, w1b, w2b, out, flag);
  return hipGetLastError();
}

hipError_t launch_stride_gather(const double* X, int64_t stride, int64_t na, double* Xa, hipStream_t s) {
  if (na <= 0) return hipSuccess;
  k_stride_gather<<<(unsigned)((na + 255) / 256), 256, 0, s>>>(X, stride, na, Xa);
  return hipGetLastError();
}

hipError_t launch_audit(const float* out, int64_t stride, int64_t na, const float* uw, double* sums,
                        hipStream_t s) {
  k_audit<<<1, 1024, 0, s>>>(out, stride, na, uw, sums);
  return hipGetLastError();
}

}  // namespace ptk
