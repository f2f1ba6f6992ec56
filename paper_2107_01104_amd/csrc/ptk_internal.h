// Internal declarations shared by the libptk translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace ptk {

constexpr int kMaxI = 8;           // largest kernel size built into the library
// Bins: tile columns of T x T cells in (x1, x2), cut along x3 into windows of
// kWindow cell layers.  T per storage type: FP32 and 16-bit nodes leave room
// for two workgroups per CU; FP64 nodes (32 bytes in LDS) fill one.
constexpr int kTileF32 = 12;       // FP32, BF16, FP16 storage
constexpr int kTileF64 = 12;       // FP64 storage
constexpr int kWindow = 5;
// windows per x3 segment of a column (one workgroup): the kernel keeps the
// segment's bin offsets in LDS
constexpr int kMaxWps = 224;
constexpr double kL = 6.283185307179586;  // fl64(2*pi)
// learned correction form: features per particle, their row pitch, parameters
constexpr int kLearnedNFeat = 195;
constexpr int kLearnedPitch = 200;
constexpr int kLearnedNParams = 41987;

// Coefficients of beta_j (val) and d beta_j / dt (der) for node index
// c = 0..I-1 (offset c - (I/2 - 1)): ascending powers of t, and (cval, cder)
// ascending powers of (t - 1/2).  The kernels evaluate the centred form: on
// [0, 1) its terms are smaller (|t - 1/2| <= 1/2), so Horner's rule in FP32
// loses far less to cancellation (for the I = 8 C2 spline's derivative the
// sum of the terms' magnitudes drops from about 42 to 4).
struct KernelTables {
  int I = 0;
  double val64[kMaxI][kMaxI];
  double der64[kMaxI][kMaxI];
  float val32[kMaxI][kMaxI];
  float der32[kMaxI][kMaxI];
  double cval64[kMaxI][kMaxI];
  double cder64[kMaxI][kMaxI];
  float cval32[kMaxI][kMaxI];
  float cder32[kMaxI][kMaxI];
};

int build_kernel_tables(int family, int I, int m, KernelTables* out);

// Geometry of the stored field: a periodic copy padded by I/2-1 nodes below
// and I/2 above on every axis, rows padded to `row_pitch` bytes.
struct FieldGeom {
  int64_t N = 0;       // grid points per axis
  int64_t P = 0;       // padded extent N + I - 1
  int64_t row_pitch = 0;    // bytes per padded x1 row
  int64_t plane_pitch = 0;  // bytes per padded (x2, x1) plane
  int node_bytes = 0;       // 3 components in the storage type
  int halo_lo = 0;          // I/2 - 1
};

// Kernel timing (ptk_timing_enable / ptk_timing_read): event pairs recorded on
// the call's stream around each instrumented launch sequence.
constexpr int kTimerKinds = 8;
struct TimedPair {
  hipEvent_t start, stop;
  int kind;
};

struct FftState;  // inverse-transform plan (spectral.hip)

// One growable device allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t cap = 0;
};

}  // namespace ptk

struct ptk_ctx {
  int device = 0;
  std::string err;
  // field
  bool has_field = false;
  int family = 0, I = 0, m = 0;
  int storage = 0;          // PTK_F64 .. PTK_F16
  float scale[3] = {1.f, 1.f, 1.f};
  ptk::FieldGeom geom;
  ptk::DevBuf field;
  // the field of the end of the next time step (same grid, kernel and
  // storage), for a Heun step whose stages see the fields of their own times
  bool has_next = false;
  ptk::FieldGeom geom_next;
  ptk::DevBuf field_next;
  float scale_next[3] = {1.f, 1.f, 1.f};
  ptk::DevBuf coef;         // device copy of the coefficient tables (KernelTables)
  ptk::KernelTables tables;
  // spectral input: transform buffer, the transform's work buffer and plan
  ptk::DevBuf spec, fft_out, fft_work;
  ptk::FftState* fft = nullptr;
  // binning of the last interpolate call
  int64_t bin_np = 0, bin_nbins = 0;
  uint32_t* bin_perm = nullptr;
  bool bin_valid = false;
  // scratch
  ptk::DevBuf keys_a, keys_b, vals_a, vals_b, offsets, hist, scan_tmp, flag;
  ptk::DevBuf xs, xn, orig, orig_b, k1, k2, gint, stage;
  ptk::DevBuf abh[4], abh_b[4];  // Adams-Bashforth history in bin order, and its permuted copy
  // incremental re-binning inside advance: sorted keys and offsets of the
  // current order (skeys, aoff) and of the next (skeys2, offsets2), mover
  // lists, per-bin counters, and the permutations of the last re-binning
  // (aperm) and of the Heun predictor's (aperm_p)
  ptk::DevBuf skeys, skeys2, aoff, offsets2, mk_a, mk_b, mv_a, mv_b, mo, rb_in, rb_out, rb_inc, rb_block;
  ptk::DevBuf aperm, aperm_p;
  // the particle state between advance calls (ptk_particles_load .. _store):
  // which buffers hold what, in the current bin order
  struct {
    bool valid = false;
    int64_t Np = 0, N = 0;
    int vb = 0;   // bytes per velocity component of the history
    int K = 0;    // history depth (Adams-Bashforth order) it was loaded for
    int hl = 0;   // valid history entries
    double* xcur = nullptr;    // positions: particle i's is row xrow[i] (row i if xrow is NULL)
    double* xnext = nullptr;   // the other position buffer
    uint32_t* xrow = nullptr;
    uint32_t* orig = nullptr;  // caller index of particle i
    uint32_t* orig_b = nullptr;
    void* k1 = nullptr;        // buffer for the next u(X_n)
    void* h[4] = {nullptr, nullptr, nullptr, nullptr};   // u_{n-1-j}
    void* hb[4] = {nullptr, nullptr, nullptr, nullptr};  // their re-binned copies
    // orientation of axisymmetric ellipsoids (Jeffery's equation), FP64, in
    // the current bin order: the unit axes, the next step's axes, the rhs of
    // the step's stages, the predictor's axes, and the rhs history
    bool ori = false;
    double shape = 0.0;
    double* p = nullptr;
    double* pn = nullptr;
    double* r1 = nullptr;
    double* r2 = nullptr;
    double* ps = nullptr;
    double* ph[4] = {nullptr, nullptr, nullptr, nullptr};
    double* phb[4] = {nullptr, nullptr, nullptr, nullptr};
    // inertial particles (dX/dt = V, dV/dt = (u - V)/tau) use the same slots
    // for V: p the velocities, pn the next step's, r1 and r2 the drag terms of
    // the stages, ps the predictor's velocities, ph the drag history; vh holds
    // the earlier velocities (the positions' Adams-Bashforth history).  A
    // particle set has axes or inertia, not both.
    bool inert = false;
    double tau = 0.0;
    double* vh[4] = {nullptr, nullptr, nullptr, nullptr};
    double* vhb[4] = {nullptr, nullptr, nullptr, nullptr};
  } adv;
  ptk::DevBuf ori_p, ori_pn, ori_r1, ori_r2, ori_ps, ori_h[4], ori_hb[4], gint2;
  ptk::DevBuf in_vh[4], in_vhb[4];  // inertial particles' velocity history and its permuted copy
  ptk::DevBuf io;  // the particle state in the caller's order, for state files
  // learned form: FP32 master parameters, Adam moments, BF16 layer copies,
  // per-workgroup gradient and loss partials, audit scratch
  ptk::DevBuf lparams, lm, lv, lw1b, lw2b, lw2bt, lgpart, llpart, lwide, laudit_x, laudit_u, laudit_sums;
  bool learned_ready = false;
  int64_t learned_step = 0;
  void* noalloc = nullptr;   // device address of the no-allocation scratch array on this device
  size_t bytes_in_use = 0;
  size_t byte_cap = 0;      // 0 = unlimited (test hook PTK_TEST_MAX_BYTES)
  bool check = true;        // PTK_NO_CHECK clears it
  // timing
  bool timing = false;
  std::vector<hipEvent_t> event_pool;
  std::vector<ptk::TimedPair> pending;
  double timer_ms[ptk::kTimerKinds] = {0};
  int64_t timer_count[ptk::kTimerKinds] = {0};
};
