// Host-side launchers of the libptk kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ptk {

// Bits of the device status word the kernels raise (atomicOr) and the host
// reads at the end of a call.
constexpr int kFlagDomain = 1;   // a position was NaN, infinite or |x| >= 2^50
constexpr int kFlagBinning = 2;  // a particle's cell lies outside its bin's tile column or window

// Bin geometry: tile columns of T x T cells in (x1, x2), ntx = ceil(N/T) per
// axis, each cut along x3 into nw = ceil(N/W) windows of W cell layers.
struct BinGeom {
  int T, ntx, W, nw;
};

// binning.hip
hipError_t launch_keys(const double* X, int64_t n, int N, double invd, const BinGeom& g, uint32_t* keys,
                       int* flag, hipStream_t s);
hipError_t launch_locate(const double* X, int64_t n3, int N, double invd, int32_t* cell, double* off,
                         int* flag, hipStream_t s);
size_t sort_hist_words(int64_t n);
size_t scan_tmp_words(int64_t m);
hipError_t exclusive_scan_u32(uint32_t* a, int64_t m, uint32_t* tmp, hipStream_t s);
hipError_t radix_sort_keys(uint32_t* ka, uint32_t* kb, uint32_t* va, uint32_t* vb, int64_t n,
                           const uint32_t* n_dev, bool vals_in_va, int key_bits, uint32_t* hist,
                           uint32_t* tmp, uint32_t** keys_sorted, uint32_t** perm, hipStream_t s);
// Stable re-sort after small moves.  okeys: the current keys, sorted, with
// CSR offsets ooff[n_bins+1]; nkeys: new keys in the same order.  Produces
// perm (new position -> current index), skeys (new sorted keys) and noff
// (new offsets); the result equals a stable sort of nkeys.  Only the
// particles whose key changed are sorted.
struct RebinScratch {
  uint32_t *in_start, *out_before, *inc_before;  // [n_bins + 1] each
  uint32_t* blockoff;                            // [n/2048 + 2]
  uint32_t *mk_a, *mk_b, *mv_a, *mv_b, *mo;      // [n] each
  uint32_t *hist, *scan_tmp;                     // as for radix_sort_keys on n elements
};
size_t rebin_block_words(int64_t n);
hipError_t rebin_incremental(const uint32_t* okeys, const uint32_t* ooff, const uint32_t* nkeys, int64_t n,
                             int64_t n_bins, int key_bits, const RebinScratch& w, uint32_t* perm, uint32_t* skeys,
                             uint32_t* noff, hipStream_t s);
hipError_t launch_fill_i32(int* p, int64_t n, int value, hipStream_t s);
hipError_t launch_offsets(const uint32_t* skeys, int64_t n, int64_t n_bins, uint32_t* offsets,
                          hipStream_t s);
hipError_t gather3_f64(const double* in, const uint32_t* perm, int64_t n, double* out, hipStream_t s);
hipError_t gather3_f32(const float* in, const uint32_t* perm, int64_t n, float* out, hipStream_t s);
hipError_t gather_u32(const uint32_t* in, const uint32_t* perm, int64_t n, uint32_t* out, hipStream_t s);
hipError_t scatter_f64(const double* in, const uint32_t* idx, int64_t n, int width, double* out,
                       hipStream_t s);
hipError_t scatter_f32(const float* in, const uint32_t* idx, int64_t n, int width, float* out,
                       hipStream_t s);

// field.hip
// A grid field in memory: component a of node (x1, x2, x3) is element
// x3*ps + x2*rs + x1*ns + a*cs (elements of the input type).
struct SrcLayout {
  int64_t cs, ns, rs, ps;
};
inline SrcLayout interleaved_layout(int64_t N) { return SrcLayout{1, 3, 3 * N, 3 * N * N}; }
// the three real planes [a][x3][x2][x1] the inverse real transform writes
inline SrcLayout transform_layout(int64_t N) { return SrcLayout{N * N * N, 1, N, N * N}; }
hipError_t launch_sumsq(const void* u, int in_f64, int64_t N, const SrcLayout& l, double* partial, int nblocks,
                        hipStream_t s);
hipError_t launch_pack(const void* u, int in_f64, const SrcLayout& l, int64_t N, int storage, int I, void* field,
                       int64_t row_pitch, int64_t plane_pitch, const float* inv_scale, hipStream_t s);
hipError_t launch_unpack(const void* field, int64_t N, int storage, int I, int64_t row_pitch, int64_t plane_pitch,
                         void* out, int out_f64, hipStream_t s);

// spectral.hip: the spectrum in transform order, and the inverse real
// transform (rocFFT) of three components into a separate real buffer
hipError_t launch_spec_prep(const void* spec, int in_f64, int64_t N, int vorticity, void* out, hipStream_t s);
struct FftState;
// (re)creates the plan for (N, precision) if needed; *work_bytes = its work buffer
int fft_prepare(FftState** st, int64_t N, int f64, size_t* work_bytes, const char** err);
int fft_run(FftState* st, void* buf, void* out, void* work, size_t work_bytes, hipStream_t s, const char** err);
void fft_release(FftState* st);

// interp.hip
struct InterpArgs {
  const void* field;
  int64_t row_pitch, plane_pitch, P;
  int N;
  double invd;
  int64_t ntx, n_tiles, nw;  // tile columns per axis, columns, x3 windows per column
  int64_t nseg, wps;         // x3 segments per column (one workgroup each), windows per segment
  const double* X;          // positions: bin-ordered particle p's is row xrow[p] (row p if xrow is NULL)
  const uint32_t* xrow;
  int64_t np;               // number of particles
  const uint32_t* offsets;  // [n_bins + 1]
  const uint32_t* orig;     // destination index of each bin-ordered particle, or NULL
  const uint32_t* grad_orig;  // destination index of its gradient row, or NULL (= orig)
  void* out;                // [n][3] or NULL
  void* grad;               // [n][3][3] or NULL
  int out_f64;
  const void* coef;         // device KernelTables
  float scale[3];
  int* flag;                // device status word (kFlag* bits)
};
hipError_t launch_interp(int storage, int I, const InterpArgs& a, hipStream_t s);

// step.hip
enum UpdateKind { kEulerOrPredict = 0, kHeunCorrect = 1, kAB = 2 };
// velocities k[j] (FP64 or FP32, [n][3], unused ones NULL) and, for kAB, the
// weights b[j] of the nk of them
struct UpdateVel {
  const void* k[4];
  double b[4];
  int nk;
};
// X: particle i's position is row xrow[i] of X (row i if xrow is NULL); Xout
// and keys are written in particle order
hipError_t launch_update(int kind, int vel_f64, const double* X, const uint32_t* xrow, const UpdateVel& v, double dt,
                         int64_t n, double* Xout, uint32_t* keys, int N, double invd, const BinGeom& g, int* flag,
                         hipStream_t s);

// orientation of axisymmetric ellipsoids (Jeffery's equation): r = rhs(G, p)
// in FP64 from the gradient G [n][3][3] (FP64 or FP32); the update of p with
// the rhs in v (FP64 [n][3] each) as launch_update does for positions, then
// normalized to unit length when `unit`
hipError_t launch_jeffery_rhs(int grad_f64, const void* G, const double* p, double shape, int64_t n, double* r,
                              hipStream_t s);
hipError_t launch_orient_update(int kind, const double* p, const UpdateVel& v, double dt, int64_t n, int unit,
                                double* out, hipStream_t s);
// inertial particles: r = (u - V) / tau (u FP64 or FP32 [n][3], V and r FP64)
hipError_t launch_drag_rhs(int vel_f64, const void* u, const double* V, double tau, int64_t n, double* r,
                           hipStream_t s);

// learned.hip
struct LearnedField {
  const void* field;  // FP32 storage, padded layout of set_field
  int64_t row_pitch, plane_pitch;
  int halo_lo;
  int N;
  double invd;
  float l4[4][4];     // Lagrange I = 4 coefficients, [node][power of t]
};
struct LearnedUpdate {
  int mode;           // 0 gradient + loss only, 1 Adam step, 2 BF16 copies only
  int nparts;         // workgroup partials to sum
  float lr, beta1, beta2, eps;
  float c1, c2;       // bias corrections 1/(1 - beta1^s), 1/(1 - beta2^s)
  float loss_scale;   // 1 / (3 batch)
  float* loss_out;    // device, one float, or NULL
  float* grad_out;    // device [kLearnedNParams] (mode 0)
};
hipError_t launch_learned_pairs(const LearnedField& f, const double* X, int64_t n, const float* uwide,
                                uint16_t* feat, float* target, int* flag, hipStream_t s);
// feat_next: the next step's batch rows (read ahead into L2), or NULL
hipError_t launch_learned_forward_backward(const uint16_t* feat, const float* target, int64_t batch,
                                           const float* params, const uint16_t* w1b, const uint16_t* w2b,
                                           const uint16_t* w2bt, float* gpart, float* lpart, hipStream_t s,
                                           const uint16_t* feat_next = nullptr);
hipError_t launch_learned_update(float* params, float* m, float* v, const float* gpart, const float* lpart,
                                 const LearnedUpdate& u, uint16_t* w1b, uint16_t* w2b, uint16_t* w2bt,
                                 hipStream_t s);
hipError_t launch_learned_infer(const LearnedField& f, const double* X, int64_t n, const uint32_t* orig,
                                const float* params, const uint16_t* w1b, const uint16_t* w2b, float* out,
                                int* flag, hipStream_t s);
hipError_t launch_stride_gather(const double* X, int64_t stride, int64_t na, double* Xa, hipStream_t s);
hipError_t launch_audit(const float* out, int64_t stride, int64_t na, const float* uw, double* sums,
                        hipStream_t s);

}  // namespace ptk
