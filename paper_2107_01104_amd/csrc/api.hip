// C ABI of libptk (declarations and contracts in include/ptk.h).
//
// Host runtime: argument validation, device scratch that grows monotonically
// (no allocation in steady state), and the sequence of kernel launches for each
// entry point, all on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <mutex>
#include <string>

#include "launch.h"
#include "ptk.h"
#include "ptk_internal.h"

using namespace ptk;

namespace {

struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != d) err = hipSetDevice(d);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int fail(ptk_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(ptk_ctx* c, hipError_t e, const char* what) {
  return fail(c, PTK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define PTK_HIP(ctx, expr, what)                 \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

#define PTK_TRY(expr)           \
  do {                          \
    int r_ = (expr);            \
    if (r_ != PTK_OK) return r_; \
  } while (0)

// Make `b` hold at least `bytes`.  The new block is allocated beside the old
// one first, so a failed growth leaves the old block (and its contents)
// intact; only when both do not fit is the old block released before a second
// attempt, and a failure then leaves `b` empty (callers whose state lives in
// the buffer, the stored field, withdraw that state before growing it).
// Releasing waits for the device, so no enqueued kernel still uses the old
// allocation when it is freed.
bool within_cap(const ptk_ctx* c, size_t extra) {
  return !c->byte_cap || c->bytes_in_use + extra <= c->byte_cap;
}

void* try_malloc(size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void drop(ptk_ctx* c, DevBuf& b) {
  if (!b.ptr) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(b.ptr);
  c->bytes_in_use -= b.cap;
  b.ptr = nullptr;
  b.cap = 0;
}

int ensure(ptk_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return PTK_OK;
  size_t want = bytes + bytes / 8;
  want = (want + 255) & ~(size_t)255;
  void* p = within_cap(c, want) ? try_malloc(want) : nullptr;
  if (!p && b.ptr) {
    drop(c, b);
    p = within_cap(c, want) ? try_malloc(want) : nullptr;
  }
  if (!p)
    return fail(c, PTK_ENOMEM,
                within_cap(c, want) ? "hipMalloc of " + std::to_string(want) + " bytes failed"
                                    : std::string("device scratch would exceed PTK_TEST_MAX_BYTES"));
  drop(c, b);
  b.ptr = p;
  b.cap = want;
  c->bytes_in_use += want;
  return PTK_OK;
}

// Host-side guard of a launch that writes `bytes` into scratch buffer `b`: an
// undersized buffer is reported as an error instead of being overrun.
int need(ptk_ctx* c, const DevBuf& b, size_t bytes, const char* what) {
  if (b.ptr && b.cap >= bytes) return PTK_OK;
  return fail(c, PTK_EINTERNAL, std::string("scratch buffer too small for ") + what);
}

void release(DevBuf& b) {
  if (b.ptr) (void)hipFree(b.ptr);
  b.ptr = nullptr;
  b.cap = 0;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

hipEvent_t take_event(ptk_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets a launch sequence with events when timing is enabled.
struct Timed {
  ptk_ctx* c;
  hipStream_t s;
  int kind;
  hipEvent_t start = nullptr;
  Timed(ptk_ctx* c_, hipStream_t s_, int k) : c(c_), s(s_), kind(k) {
    if (!c->timing) return;
    start = take_event(c);
    if (start && hipEventRecord(start, s) != hipSuccess) {
      c->event_pool.push_back(start);
      start = nullptr;
    }
  }
  ~Timed() {
    if (!start) return;
    hipEvent_t stop = take_event(c);
    if (stop && hipEventRecord(stop, s) == hipSuccess) {
      c->pending.push_back(TimedPair{start, stop, kind});
    } else {
      c->event_pool.push_back(start);
      if (stop) c->event_pool.push_back(stop);
    }
  }
};

// Waits for the recorded pairs and folds them into the accumulators.
void drain_timers(ptk_ctx* c) {
  for (TimedPair& p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      c->timer_ms[p.kind] += ms;
      c->timer_count[p.kind] += 1;
    }
    c->event_pool.push_back(p.start);
    c->event_pool.push_back(p.stop);
  }
  c->pending.clear();
}

BinGeom bin_geom(const ptk_ctx* c) {
  BinGeom g;
  g.T = c->storage == PTK_F64 ? kTileF64 : kTileF32;
  g.ntx = (int)((c->geom.N + g.T - 1) / g.T);
  g.W = kWindow;
  g.nw = (int)((c->geom.N + g.W - 1) / g.W);
  return g;
}

inline int64_t n_bins_of(const BinGeom& g) { return (int64_t)g.ntx * g.ntx * g.nw; }

inline int bits_for(int64_t n_bins) {
  int b = 0;
  while (((int64_t)1 << b) < n_bins) ++b;
  return b;
}

inline double invd_of(int64_t N) { return (double)N / kL; }

int vel_bytes(const ptk_ctx* c) { return c->storage == PTK_F64 ? 8 : 4; }

int flag_error(ptk_ctx* c, int h) {
  if (h & kFlagDomain) return fail(c, PTK_EDOMAIN, "a particle position is NaN, infinite or has |x| >= 2^50");
  if (h & kFlagBinning)
    return fail(c, PTK_EINTERNAL, "a particle's cell lies outside the tile column or window of its bin");
  return PTK_OK;
}

int check_flag(ptk_ctx* c, hipStream_t s) {
  if (!c->check) return PTK_OK;
  int h = 0;
  PTK_HIP(c, hipMemcpyAsync(&h, c->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s), "flag read");
  PTK_HIP(c, hipStreamSynchronize(s), "stream synchronize");
  return flag_error(c, h);
}

// scratch for binning Np particles over n_bins bins
int ensure_binning(ptk_ctx* c, int64_t Np, int64_t n_bins) {
  const size_t n4 = (size_t)Np * 4;
  PTK_TRY(ensure(c, c->keys_a, n4));
  PTK_TRY(ensure(c, c->keys_b, n4));
  PTK_TRY(ensure(c, c->vals_a, n4));
  PTK_TRY(ensure(c, c->vals_b, n4));
  const size_t hw = sort_hist_words(Np);
  PTK_TRY(ensure(c, c->hist, hw * 4));
  const int64_t scan_max = (int64_t)hw > n_bins + 1 ? (int64_t)hw : n_bins + 1;
  PTK_TRY(ensure(c, c->scan_tmp, scan_tmp_words(scan_max) * 4));
  PTK_TRY(ensure(c, c->offsets, (size_t)(n_bins + 1) * 4));
  return PTK_OK;
}

// scratch of the incremental re-binning (in addition to ensure_binning's)
int ensure_rebin(ptk_ctx* c, int64_t Np, int64_t n_bins) {
  const size_t n4 = (size_t)Np * 4, b4 = (size_t)(n_bins + 1) * 4;
  DevBuf* per_particle[] = {&c->skeys, &c->skeys2, &c->mk_a, &c->mk_b, &c->mv_a, &c->mv_b, &c->mo,
                            &c->aperm, &c->aperm_p};
  for (DevBuf* b : per_particle) PTK_TRY(ensure(c, *b, n4));
  DevBuf* per_bin[] = {&c->aoff, &c->offsets2, &c->rb_in, &c->rb_out, &c->rb_inc};
  for (DevBuf* b : per_bin) PTK_TRY(ensure(c, *b, b4));
  PTK_TRY(ensure(c, c->rb_block, rebin_block_words(Np) * 4));
  return PTK_OK;
}

// Host-side checks that the scratch a launch sequence writes is as large as
// the launches assume (the ensure calls grow it; these catch a growth that a
// code path forgot, as an error code instead of an out-of-bounds write).
int check_binning_caps(ptk_ctx* c, int64_t Np, int64_t n_bins) {
  const size_t n4 = (size_t)Np * 4;
  PTK_TRY(need(c, c->keys_a, n4, "bin keys"));
  PTK_TRY(need(c, c->keys_b, n4, "bin keys"));
  PTK_TRY(need(c, c->vals_a, n4, "sort values"));
  PTK_TRY(need(c, c->vals_b, n4, "sort values"));
  const size_t hw = sort_hist_words(Np);
  PTK_TRY(need(c, c->hist, hw * 4, "sort histograms"));
  const int64_t scan_max = (int64_t)hw > n_bins + 1 ? (int64_t)hw : n_bins + 1;
  PTK_TRY(need(c, c->scan_tmp, scan_tmp_words(scan_max) * 4, "scan partials"));
  PTK_TRY(need(c, c->offsets, (size_t)(n_bins + 1) * 4, "bin offsets"));
  return PTK_OK;
}

int check_rebin_caps(ptk_ctx* c, int64_t Np, int64_t n_bins) {
  const size_t n4 = (size_t)Np * 4, b4 = (size_t)(n_bins + 1) * 4;
  const DevBuf* per_particle[] = {&c->skeys, &c->skeys2, &c->mk_a, &c->mk_b, &c->mv_a, &c->mv_b, &c->mo,
                                  &c->aperm, &c->aperm_p};
  for (const DevBuf* b : per_particle) PTK_TRY(need(c, *b, n4, "re-binning lists"));
  const DevBuf* per_bin[] = {&c->aoff, &c->offsets2, &c->rb_in, &c->rb_out, &c->rb_inc};
  for (const DevBuf* b : per_bin) PTK_TRY(need(c, *b, b4, "re-binning offsets"));
  PTK_TRY(need(c, c->rb_block, rebin_block_words(Np) * 4, "re-binning block offsets"));
  return PTK_OK;
}

// keys -> stable sort -> offsets.  keys of the particles must be in keys_a.
// *skeys (optional) receives the sorted keys' location.
int bin_sorted(ptk_ctx* c, int64_t Np, int64_t n_bins, uint32_t** perm, hipStream_t s,
               uint32_t** skeys = nullptr, uint32_t* off_out = nullptr) {
  uint32_t* sk = nullptr;
  PTK_HIP(c,
          radix_sort_keys((uint32_t*)c->keys_a.ptr, (uint32_t*)c->keys_b.ptr, (uint32_t*)c->vals_a.ptr,
                          (uint32_t*)c->vals_b.ptr, Np, nullptr, false, bits_for(n_bins), (uint32_t*)c->hist.ptr,
                          (uint32_t*)c->scan_tmp.ptr, &sk, perm, s),
          "radix sort");
  PTK_HIP(c, launch_offsets(sk, Np, n_bins, off_out ? off_out : (uint32_t*)c->offsets.ptr, s), "bin offsets");
  if (skeys) *skeys = sk;
  return PTK_OK;
}

InterpArgs base_args(const ptk_ctx* c, bool next_field = false) {
  InterpArgs a;
  std::memset(&a, 0, sizeof(a));
  const BinGeom g = bin_geom(c);
  a.field = next_field ? c->field_next.ptr : c->field.ptr;
  a.row_pitch = c->geom.row_pitch;
  a.plane_pitch = c->geom.plane_pitch;
  a.P = c->geom.P;
  a.N = (int)c->geom.N;
  a.invd = invd_of(c->geom.N);
  a.ntx = g.ntx;
  a.n_tiles = (int64_t)g.ntx * g.ntx;
  a.nw = g.nw;
  // enough workgroups to fill the GPU: split columns along x3 when there are few
  int64_t nseg = (1024 + a.n_tiles - 1) / a.n_tiles;
  if (nseg > a.nw) nseg = a.nw;
  if (nseg < 1) nseg = 1;
  if (nseg < (a.nw + kMaxWps - 1) / kMaxWps) nseg = (a.nw + kMaxWps - 1) / kMaxWps;
  a.wps = (a.nw + nseg - 1) / nseg;
  a.nseg = (a.nw + a.wps - 1) / a.wps;
  a.offsets = (const uint32_t*)c->offsets.ptr;
  a.coef = c->coef.ptr;
  a.flag = (int*)c->flag.ptr;
  for (int q = 0; q < 3; ++q) a.scale[q] = next_field ? c->scale_next[q] : c->scale[q];
  return a;
}

// Device scratch of one interpolate call: sort keys and values (double
// buffered), radix histograms, scan partials, bin offsets.
struct InterpScratch {
  uint32_t *keys_a, *keys_b, *vals_a, *vals_b, *hist, *scan_tmp, *offsets;
};

int check_interp_args(ptk_ctx* c, const double* X, int64_t Np, void* u_out, void* grad, int out_dtype) {
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (Np < 0 || Np > (int64_t)0xFFFFFFFF) return fail(c, PTK_EINVAL, "Np out of range [0, 2^32)");
  if (out_dtype != PTK_F64 && out_dtype != PTK_F32) return fail(c, PTK_EINVAL, "out_dtype must be F64 or F32");
  if (Np > 0 && (!X || (!u_out && !grad))) return fail(c, PTK_EINVAL, "NULL pointer");
  return PTK_OK;
}

// keys -> stable sort -> offsets -> interpolation kernel, on the given
// scratch; records the binning when `record` (the scratch then stays the
// context's until the next call).  Arguments are checked by the caller and
// the device is current.
int interp_core(ptk_ctx* c, const InterpScratch& w, const double* X, int64_t Np, void* u_out, void* grad,
                int out_dtype, hipStream_t s, bool record) {
  const int64_t N = c->geom.N;
  const BinGeom bg = bin_geom(c);
  const int64_t n_bins = n_bins_of(bg);
  c->bin_valid = false;
  if (Np == 0) {
    PTK_HIP(c, launch_offsets(w.keys_a, 0, n_bins, w.offsets, s), "bin offsets");
    if (record) {
      c->bin_np = 0;
      c->bin_nbins = n_bins;
      c->bin_perm = nullptr;
      c->bin_valid = true;
    }
    return PTK_OK;
  }
  PTK_HIP(c, launch_fill_i32((int*)c->flag.ptr, 1, 0, s), "flag clear");
  {
    Timed t(c, s, PTK_T_KEYS);
    PTK_HIP(c, launch_keys(X, Np, (int)N, invd_of(N), bg, w.keys_a, (int*)c->flag.ptr, s), "keys");
  }
  uint32_t* perm = nullptr;
  {
    Timed t(c, s, PTK_T_SORT);
    uint32_t* sk = nullptr;
    PTK_HIP(c,
            radix_sort_keys(w.keys_a, w.keys_b, w.vals_a, w.vals_b, Np, nullptr, false, bits_for(n_bins), w.hist,
                            w.scan_tmp, &sk, &perm, s),
            "radix sort");
    PTK_HIP(c, launch_offsets(sk, Np, n_bins, w.offsets, s), "bin offsets");
  }
  // the kernel reads the caller's positions through the bin permutation (the
  // order it also writes the results in): no gathered copy
  InterpArgs a = base_args(c);
  a.offsets = w.offsets;
  a.X = X;
  a.xrow = perm;
  a.np = Np;
  a.orig = perm;
  a.out = u_out;
  a.grad = grad;
  a.out_f64 = out_dtype == PTK_F64;
  {
    Timed t(c, s, grad ? PTK_T_INTERP_GRAD : PTK_T_INTERP);
    PTK_HIP(c, launch_interp(c->storage, c->I, a, s), "interpolate");
  }
  if (record) {
    c->bin_perm = perm;
    c->bin_np = Np;
    c->bin_nbins = n_bins;
    c->bin_valid = true;
  }
  return check_flag(c, s);
}

int interp_common(ptk_ctx* c, const double* X, int64_t Np, void* u_out, void* grad, int out_dtype,
                  void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  PTK_TRY(check_interp_args(c, X, Np, u_out, grad, out_dtype));
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  const int64_t n_bins = n_bins_of(bin_geom(c));
  c->bin_valid = false;
  if (Np == 0) {
    PTK_TRY(ensure(c, c->offsets, (size_t)(n_bins + 1) * 4));
  } else {
    PTK_TRY(ensure_binning(c, Np, n_bins));
    PTK_TRY(check_binning_caps(c, Np, n_bins));
  }
  PTK_TRY(need(c, c->offsets, (size_t)(n_bins + 1) * 4, "bin offsets"));
  InterpScratch w{(uint32_t*)c->keys_a.ptr, (uint32_t*)c->keys_b.ptr, (uint32_t*)c->vals_a.ptr,
                  (uint32_t*)c->vals_b.ptr,  (uint32_t*)c->hist.ptr,   (uint32_t*)c->scan_tmp.ptr,
                  (uint32_t*)c->offsets.ptr};
  return interp_core(c, w, X, Np, u_out, grad, out_dtype, S(stream), true);
}

// ---- the no-allocation entry point's scratch: one array per GPU, in the
// library's code object (the loader places a copy on every device the
// library runs on; it lives until the process ends).  Host code uses only the
// device address hipGetSymbolAddress reports for the current device, never
// the array's name.
constexpr size_t kNoAllocBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// The device address of `scratch` on the current device `device`, looked up
// once per device (at ptk_create); NULL on failure.
void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    g_scratch_ptr[device] = p;
    g_scratch_done[device] = true;
  }
  return g_scratch_ptr[device];
}

// Carve an interpolate call's scratch out of `base` (kNoAllocBytes); false
// if it does not fit.
bool carve_noalloc(unsigned char* base, int64_t Np, int64_t n_bins, InterpScratch* w, size_t* need_bytes) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return (uint32_t*)p;
  };
  const size_t n4 = (size_t)(Np > 0 ? Np : 1) * 4;
  w->keys_a = take(n4);
  w->keys_b = take(n4);
  w->vals_a = take(n4);
  w->vals_b = take(n4);
  const size_t hw = sort_hist_words(Np);
  w->hist = take(hw * 4);
  const int64_t scan_max = (int64_t)hw > n_bins + 1 ? (int64_t)hw : n_bins + 1;
  w->scan_tmp = take(scan_tmp_words(scan_max) * 4);
  w->offsets = take((size_t)(n_bins + 1) * 4);
  *need_bytes = off;
  return off <= kNoAllocBytes;
}

// ---- learned form helpers
int learned_field(ptk_ctx* c, LearnedField* lf) {
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (c->storage != PTK_F32) return fail(c, PTK_EUNSUPPORTED, "the learned form needs FP32 field storage");
  KernelTables t4;
  if (build_kernel_tables(PTK_LAGRANGE, 4, 0, &t4) != 0) return fail(c, PTK_EINVAL, "L4 table");
  lf->field = c->field.ptr;
  lf->row_pitch = c->geom.row_pitch;
  lf->plane_pitch = c->geom.plane_pitch;
  lf->halo_lo = c->geom.halo_lo;
  lf->N = (int)c->geom.N;
  lf->invd = invd_of(c->geom.N);
  for (int j = 0; j < 4; ++j)
    for (int p = 0; p < 4; ++p) lf->l4[j][p] = t4.val32[j][p];
  return PTK_OK;
}

constexpr int kLearnedMaxBatch = 16384;

int check_rows(ptk_ctx* c, const uint16_t* feat, const float* target, int64_t n) {
  if (!c->learned_ready) return fail(c, PTK_EINVAL, "no network parameters set");
  if (!feat || !target) return fail(c, PTK_EINVAL, "NULL pointer");
  if (((uintptr_t)feat & 15) != 0) return fail(c, PTK_EINVAL, "feature rows must be 16-byte aligned");
  (void)n;
  return PTK_OK;
}

int ensure_partials(ptk_ctx* c, int64_t batch) {
  const int64_t parts = batch / 64;
  PTK_TRY(ensure(c, c->lgpart, (size_t)parts * kLearnedNParams * 4));
  PTK_TRY(ensure(c, c->llpart, (size_t)parts * 4));
  PTK_TRY(need(c, c->lgpart, (size_t)parts * kLearnedNParams * 4, "gradient partials"));
  PTK_TRY(need(c, c->llpart, (size_t)parts * 4, "loss partials"));
  return PTK_OK;
}

}  // namespace

extern "C" {

int ptk_kernel_table(const ptk_kernel* k, double* val, double* der) {
  if (!k || !val) return PTK_EINVAL;
  if (k->family != PTK_LAGRANGE && k->family != PTK_SPLINE) return PTK_EINVAL;
  if (k->I % 2 != 0) return PTK_EUNSUPPORTED;
  if (k->I != 4 && k->I != 6 && k->I != 8) return PTK_EUNSUPPORTED;
  const int m = k->family == PTK_LAGRANGE ? 0 : k->m;
  if (m < 0 || m > k->I / 2 - 1) return PTK_EINVAL;
  KernelTables tab;
  int r = build_kernel_tables(k->family, k->I, m, &tab);
  if (r != 0) return r == -6 ? PTK_EUNSUPPORTED : PTK_EINVAL;
  for (int j = 0; j < k->I; ++j)
    for (int p = 0; p < k->I; ++p) {
      val[j * k->I + p] = tab.val64[j][p];
      if (der) der[j * k->I + p] = tab.der64[j][p];
    }
  return PTK_OK;
}

int ptk_kernel_table_centred(const ptk_kernel* k, double* val, double* der, float* val32, float* der32) {
  if (!k || !val) return PTK_EINVAL;
  if (k->family != PTK_LAGRANGE && k->family != PTK_SPLINE) return PTK_EINVAL;
  if (k->I % 2 != 0) return PTK_EUNSUPPORTED;
  if (k->I != 4 && k->I != 6 && k->I != 8) return PTK_EUNSUPPORTED;
  const int m = k->family == PTK_LAGRANGE ? 0 : k->m;
  if (m < 0 || m > k->I / 2 - 1) return PTK_EINVAL;
  KernelTables tab;
  int r = build_kernel_tables(k->family, k->I, m, &tab);
  if (r != 0) return r == -6 ? PTK_EUNSUPPORTED : PTK_EINVAL;
  for (int j = 0; j < k->I; ++j)
    for (int p = 0; p < k->I; ++p) {
      val[j * k->I + p] = tab.cval64[j][p];
      if (der) der[j * k->I + p] = tab.cder64[j][p];
      if (val32) val32[j * k->I + p] = tab.cval32[j][p];
      if (der32) der32[j * k->I + p] = tab.cder32[j][p];
    }
  return PTK_OK;
}

int ptk_create(ptk_ctx** out, int device) {
  if (!out) return PTK_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PTK_EINVAL;
  ptk_ctx* c = new (std::nothrow) ptk_ctx();
  if (!c) return PTK_ENOMEM;
  c->device = device;
  if (const char* cap = std::getenv("PTK_TEST_MAX_BYTES")) c->byte_cap = (size_t)std::strtoull(cap, nullptr, 10);
  if (const char* nc = std::getenv("PTK_NO_CHECK")) c->check = !(nc[0] == '1');
  DeviceGuard g(device);
  if (g.err != hipSuccess) {
    delete c;
    return PTK_EHIP;
  }
  int r = ensure(c, c->flag, 256);
  if (r != PTK_OK) {
    delete c;
    return r;
  }
  c->noalloc = noalloc_scratch(device);
  *out = c;
  return PTK_OK;
}

void ptk_destroy(ptk_ctx* c) {
  if (!c) return;
  {
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    DevBuf* bufs[] = {&c->field, &c->field_next, &c->coef, &c->keys_a, &c->keys_b, &c->vals_a, &c->vals_b, &c->offsets,
                      &c->hist, &c->scan_tmp, &c->flag, &c->xs, &c->xn, &c->orig, &c->orig_b, &c->k1,
                      &c->k2, &c->abh[0], &c->abh[1], &c->abh[2], &c->abh[3], &c->abh_b[0], &c->abh_b[1],
                      &c->abh_b[2], &c->abh_b[3], &c->gint, &c->stage, &c->lparams,
                      &c->lm, &c->lv, &c->lw1b, &c->lw2b, &c->lw2bt, &c->lgpart, &c->llpart, &c->lwide,
                      &c->laudit_x, &c->laudit_u, &c->laudit_sums, &c->skeys, &c->skeys2, &c->offsets2,
                      &c->mk_a, &c->mk_b, &c->mv_a, &c->mv_b, &c->mo, &c->rb_in, &c->rb_out, &c->rb_inc,
                      &c->rb_block, &c->spec, &c->fft_out, &c->fft_work, &c->aoff, &c->aperm, &c->aperm_p,
                      &c->ori_p, &c->ori_pn, &c->ori_r1, &c->ori_r2, &c->ori_ps, &c->ori_h[0], &c->ori_h[1],
                      &c->ori_h[2], &c->ori_h[3], &c->ori_hb[0], &c->ori_hb[1], &c->ori_hb[2], &c->ori_hb[3],
                      &c->gint2, &c->io};
    for (DevBuf* b : bufs) release(*b);
    fft_release(c->fft);
    c->fft = nullptr;
    for (TimedPair& p : c->pending) {
      (void)hipEventDestroy(p.start);
      (void)hipEventDestroy(p.stop);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  }
  delete c;
}

const char* ptk_last_error(const ptk_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

namespace {

// Checks of the arguments ptk_set_field and ptk_set_field_spectral share; the
// kernel tables come out.
int check_field_args(ptk_ctx* c, int64_t N, int in_dtype, int storage_dtype, const ptk_kernel* k,
                     KernelTables* tab, int* m_out) {
  if (N < 8 || N > 4096) return fail(c, PTK_EINVAL, "N must be in [8, 4096]");
  if (in_dtype != PTK_F64 && in_dtype != PTK_F32) return fail(c, PTK_EINVAL, "in_dtype must be F64 or F32");
  if (storage_dtype < PTK_F64 || storage_dtype > PTK_F16) return fail(c, PTK_EINVAL, "bad storage dtype");
  if (k->family != PTK_LAGRANGE && k->family != PTK_SPLINE) return fail(c, PTK_EINVAL, "bad kernel family");
  if (k->I % 2 != 0) return fail(c, PTK_EUNSUPPORTED, "odd kernel sizes are not defined");
  if (k->I != 4 && k->I != 6 && k->I != 8) return fail(c, PTK_EUNSUPPORTED, "kernel size I must be 4, 6 or 8");
  const int m = k->family == PTK_LAGRANGE ? 0 : k->m;
  if (m < 0 || m > k->I / 2 - 1) return fail(c, PTK_EINVAL, "smoothness m must be in [0, I/2-1]");
  int tr = build_kernel_tables(k->family, k->I, m, tab);
  if (tr != 0) return fail(c, tr == -6 ? PTK_EUNSUPPORTED : PTK_EINVAL, "kernel table construction failed");
  *m_out = m;
  return PTK_OK;
}

// Stores the grid field u (layout l, FP64 or FP32) as the context's field:
// the per-component scale for 16-bit storage, the coefficient tables, the pack.
int store_field(ptk_ctx* c, const void* u, int in_f64, const SrcLayout& l, int64_t N, int storage_dtype,
                const ptk_kernel* k, int m, const KernelTables& tab, hipStream_t s, bool next_field = false) {
  FieldGeom geo;
  geo.N = N;
  geo.P = N + k->I - 1;
  geo.node_bytes = storage_dtype == PTK_F64 ? 24 : storage_dtype == PTK_F32 ? 12 : 6;
  geo.halo_lo = k->I / 2 - 1;
  geo.row_pitch = ((geo.P * geo.node_bytes + 48) + 63) / 64 * 64;
  geo.plane_pitch = geo.row_pitch * geo.P;
  const size_t field_bytes = (size_t)(geo.plane_pitch * geo.P) + 64;

  // per-component scale for 16-bit storage
  float inv[3] = {1.f, 1.f, 1.f}, scl[3] = {1.f, 1.f, 1.f};
  const int64_t nodes = N * N * N;
  if (storage_dtype == PTK_BF16 || storage_dtype == PTK_F16) {
    const int nblk = 1024;
    PTK_TRY(ensure(c, c->stage, (size_t)nblk * 3 * sizeof(double)));
    PTK_TRY(need(c, c->stage, (size_t)nblk * 3 * sizeof(double), "sum-of-squares partials"));
    PTK_HIP(c, launch_sumsq(u, in_f64, N, l, (double*)c->stage.ptr, nblk, s), "sum of squares");
    double* part = new (std::nothrow) double[nblk * 3];
    if (!part) return fail(c, PTK_ENOMEM, "host allocation failed");
    hipError_t e = hipMemcpyAsync(part, c->stage.ptr, sizeof(double) * nblk * 3, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      delete[] part;
      return hip_fail(c, e, "scale read-back");
    }
    for (int q = 0; q < 3; ++q) {
      double sum = 0.0;
      for (int b = 0; b < nblk; ++b) sum += part[3 * b + q];
      const double rms = std::sqrt(sum / (double)nodes);
      if (!(rms > 0.0) || !std::isfinite(rms)) {
        delete[] part;
        return fail(c, PTK_EINVAL, "a field component is zero or not finite: cannot scale to unit rms");
      }
      inv[q] = (float)(1.0 / rms);
      scl[q] = (float)rms;
    }
    delete[] part;
  }
  if (next_field) {
    // the next time's field: same kernel, tables and storage as the current
    c->has_next = false;
    PTK_TRY(ensure(c, c->field_next, field_bytes));
    PTK_TRY(need(c, c->field_next, field_bytes, "stored next field"));
    PTK_HIP(c,
            launch_pack(u, in_f64, l, N, storage_dtype, k->I, c->field_next.ptr, geo.row_pitch, geo.plane_pitch, inv,
                        s),
            "field pack");
    c->geom_next = geo;
    for (int q = 0; q < 3; ++q) c->scale_next[q] = scl[q];
    c->has_next = true;
    return PTK_OK;
  }
  // the stored field is withdrawn while its buffer is replaced and filled: a
  // failure below leaves the context without a field (PTK_ENOFIELD), never
  // with a released or half-written one
  c->has_field = false;
  c->has_next = false;  // a new current field retires the next one
  c->bin_valid = false;
  PTK_TRY(ensure(c, c->field, field_bytes));
  PTK_TRY(ensure(c, c->coef, sizeof(KernelTables)));
  PTK_TRY(need(c, c->field, field_bytes, "stored field"));
  PTK_TRY(need(c, c->coef, sizeof(KernelTables), "coefficient tables"));
  c->tables = tab;
  PTK_HIP(c, hipMemcpyAsync(c->coef.ptr, &c->tables, sizeof(KernelTables), hipMemcpyHostToDevice, s),
          "coefficient upload");
  PTK_HIP(c, launch_pack(u, in_f64, l, N, storage_dtype, k->I, c->field.ptr, geo.row_pitch, geo.plane_pitch, inv, s),
          "field pack");
  c->geom = geo;
  c->family = k->family;
  c->I = k->I;
  c->m = m;
  c->storage = storage_dtype;
  for (int q = 0; q < 3; ++q) c->scale[q] = scl[q];
  c->has_field = true;
  c->bin_valid = false;
  return PTK_OK;
}

}  // namespace

namespace {

// The grid field of a half spectrum (velocity, or vorticity through the
// Biot-Savart law) into c->fft_out: the three real planes [a][x3][x2][x1].
int spectrum_to_grid(ptk_ctx* c, const void* spec, int64_t N, int f64, int kind, hipStream_t s) {
  const size_t rb = f64 ? 8 : 4;
  const size_t modes = (size_t)N * (size_t)N * (size_t)(N / 2 + 1);
  size_t work = 0;
  const char* msg = nullptr;
  if (fft_prepare(&c->fft, N, f64, &work, &msg) != 0) return fail(c, PTK_EHIP, msg);
  PTK_TRY(ensure(c, c->spec, 3 * modes * 2 * rb));
  PTK_TRY(ensure(c, c->fft_out, 3 * (size_t)N * (size_t)N * (size_t)N * rb));
  if (work > 0) PTK_TRY(ensure(c, c->fft_work, work));
  PTK_TRY(need(c, c->spec, 3 * modes * 2 * rb, "transform input"));
  PTK_TRY(need(c, c->fft_out, 3 * (size_t)N * (size_t)N * (size_t)N * rb, "transform output"));
  if (work > 0) PTK_TRY(need(c, c->fft_work, work, "transform work"));
  Timed t(c, s, PTK_T_IFT);
  PTK_HIP(c, launch_spec_prep(spec, f64, N, kind == PTK_SPEC_VORTICITY, c->spec.ptr, s), "spectrum prep");
  if (fft_run(c->fft, c->spec.ptr, c->fft_out.ptr, c->fft_work.ptr, c->fft_work.cap, s, &msg) != 0)
    return fail(c, PTK_EHIP, msg);
  return PTK_OK;
}

}  // namespace

int ptk_set_field(ptk_ctx* c, const void* u, int64_t N, int in_dtype, int storage_dtype, const ptk_kernel* k,
                  void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!u || !k) return fail(c, PTK_EINVAL, "NULL pointer");
  KernelTables tab;
  int m = 0;
  PTK_TRY(check_field_args(c, N, in_dtype, storage_dtype, k, &tab, &m));
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  return store_field(c, u, in_dtype == PTK_F64, interleaved_layout(N), N, storage_dtype, k, m, tab, S(stream));
}

int ptk_set_field_spectral(ptk_ctx* c, const void* spec, int64_t N, int in_dtype, int kind, int storage_dtype,
                           const ptk_kernel* k, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!spec || !k) return fail(c, PTK_EINVAL, "NULL pointer");
  if (kind != PTK_SPEC_VELOCITY && kind != PTK_SPEC_VORTICITY) return fail(c, PTK_EINVAL, "bad spectrum kind");
  if (N % 2 != 0) return fail(c, PTK_EINVAL, "N must be even for a half spectrum");
  if (N > 2048) return fail(c, PTK_EINVAL, "N must be at most 2048 for a spectral field");
  KernelTables tab;
  int m = 0;
  PTK_TRY(check_field_args(c, N, in_dtype, storage_dtype, k, &tab, &m));
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int f64 = in_dtype == PTK_F64;
  PTK_TRY(spectrum_to_grid(c, spec, N, f64, kind, s));
  return store_field(c, c->fft_out.ptr, f64, transform_layout(N), N, storage_dtype, k, m, tab, s);
}

int ptk_set_field_next(ptk_ctx* c, const void* src, int64_t N, int in_dtype, int form, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!src) return fail(c, PTK_EINVAL, "NULL pointer");
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no current field: set one with ptk_set_field first");
  if (form != PTK_GRID && form != PTK_SPEC_VELOCITY && form != PTK_SPEC_VORTICITY)
    return fail(c, PTK_EINVAL, "form must be PTK_GRID, PTK_SPEC_VELOCITY or PTK_SPEC_VORTICITY");
  if (in_dtype != PTK_F64 && in_dtype != PTK_F32) return fail(c, PTK_EINVAL, "in_dtype must be F64 or F32");
  if (N != c->geom.N) return fail(c, PTK_EINVAL, "the next field must have the current field's N");
  if (form != PTK_GRID && (N % 2 != 0 || N > 2048))
    return fail(c, PTK_EINVAL, "a spectral field needs an even N of at most 2048");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const ptk_kernel k{c->family, c->I, c->m};
  const int f64 = in_dtype == PTK_F64;
  if (form == PTK_GRID)
    return store_field(c, src, f64, interleaved_layout(N), N, c->storage, &k, c->m, c->tables, s, true);
  PTK_TRY(spectrum_to_grid(c, src, N, f64, form, s));
  return store_field(c, c->fft_out.ptr, f64, transform_layout(N), N, c->storage, &k, c->m, c->tables, s, true);
}

int ptk_get_field(ptk_ctx* c, void* u, int out_dtype, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (!u) return fail(c, PTK_EINVAL, "NULL pointer");
  if (out_dtype != PTK_F64 && out_dtype != PTK_F32) return fail(c, PTK_EINVAL, "out_dtype must be F64 or F32");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  PTK_HIP(c,
          launch_unpack(c->field.ptr, c->geom.N, c->storage, c->I, c->geom.row_pitch, c->geom.plane_pitch, u,
                        out_dtype == PTK_F64, S(stream)),
          "field unpack");
  return PTK_OK;
}

int ptk_get_field_scale(const ptk_ctx* c, float* scale3) {
  if (!c || !scale3) return PTK_EINVAL;
  if (!c->has_field) return PTK_ENOFIELD;
  for (int q = 0; q < 3; ++q) scale3[q] = c->scale[q];
  return PTK_OK;
}

int ptk_locate(ptk_ctx* c, const double* X, int64_t Np, int32_t* cell, double* t, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (Np < 0 || Np > ((int64_t)1 << 40)) return fail(c, PTK_EINVAL, "Np out of range");
  if (Np > 0 && (!X || !cell)) return fail(c, PTK_EINVAL, "NULL pointer");
  if (Np == 0) return PTK_OK;
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  PTK_HIP(c, launch_fill_i32((int*)c->flag.ptr, 1, 0, s), "flag clear");
  PTK_HIP(c, launch_locate(X, 3 * Np, (int)c->geom.N, invd_of(c->geom.N), cell, t, (int*)c->flag.ptr, s),
          "locate");
  return check_flag(c, s);
}

int ptk_interpolate(ptk_ctx* c, const double* X, int64_t Np, void* out, int out_dtype, void* stream) {
  if (c && Np > 0 && !out) return fail(c, PTK_EINVAL, "NULL output");
  return interp_common(c, X, Np, out, nullptr, out_dtype, stream);
}

int ptk_interpolate_gradient(ptk_ctx* c, const double* X, int64_t Np, void* u_out, void* grad, int out_dtype,
                             void* stream) {
  if (c && Np > 0 && !grad) return fail(c, PTK_EINVAL, "NULL gradient output");
  return interp_common(c, X, Np, u_out, grad, out_dtype, stream);
}

int ptk_interpolate_noalloc(ptk_ctx* c, const double* X, int64_t Np, void* out, int out_dtype, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (Np > 0 && !out) return fail(c, PTK_EINVAL, "NULL output");
  PTK_TRY(check_interp_args(c, X, Np, out, nullptr, out_dtype));
  if (!c->noalloc) return fail(c, PTK_EHIP, "the device address of the library's scratch array is unknown");
  const int64_t n_bins = n_bins_of(bin_geom(c));
  InterpScratch w;
  size_t need_bytes = 0;
  if (!carve_noalloc((unsigned char*)c->noalloc, Np, n_bins, &w, &need_bytes))
    return fail(c, PTK_EINVAL,
                "the call needs " + std::to_string(need_bytes) + " bytes of scratch, more than the " +
                    std::to_string(kNoAllocBytes) + " of the no-allocation array");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  return interp_core(c, w, X, Np, out, nullptr, out_dtype, S(stream), false);
}

int ptk_binning_info(const ptk_ctx* c, int64_t* np, int64_t* n_bins, int* tile, int* window) {
  if (!c || !np || !n_bins || !tile || !window) return PTK_EINVAL;
  if (!c->bin_valid) return PTK_ENOFIELD;
  const BinGeom g = bin_geom(c);
  *np = c->bin_np;
  *n_bins = c->bin_nbins;
  *tile = g.T;
  *window = g.W;
  return PTK_OK;
}

int ptk_get_binning(ptk_ctx* c, uint32_t* perm, uint32_t* offsets, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->bin_valid) return fail(c, PTK_ENOFIELD, "no binning recorded");
  if ((c->bin_np > 0 && !perm) || !offsets) return fail(c, PTK_EINVAL, "NULL pointer");
  DeviceGuard g(c->device);
  hipStream_t s = S(stream);
  if (c->bin_np > 0)
    PTK_HIP(c, hipMemcpyAsync(perm, c->bin_perm, (size_t)c->bin_np * 4, hipMemcpyDeviceToDevice, s), "copy perm");
  PTK_HIP(c,
          hipMemcpyAsync(offsets, c->offsets.ptr, (size_t)(c->bin_nbins + 1) * 4, hipMemcpyDeviceToDevice, s),
          "copy offsets");
  return PTK_OK;
}

namespace {

// Adams-Bashforth order of a scheme (0: not a multistep scheme)
int ab_order(int scheme) { return scheme == PTK_AB2 ? 2 : scheme == PTK_AB3 ? 3 : scheme == PTK_AB4 ? 4 : 0; }

// Adams-Bashforth weights of u_{n-j} by order (order 1 is Euler)
const double kABW[5][4] = {{0, 0, 0, 0},
                           {1.0, 0, 0, 0},
                           {1.5, -0.5, 0, 0},
                           {23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0, 0},
                           {55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0}};

// Sorts the caller's particles into bin order and makes them the loaded
// state: positions gathered into xs, caller index into orig, the hl valid
// history entries of rhs_hist ([K][Np][3], caller order) gathered, the bins'
// sorted keys and offsets in skeys / aoff.  Argument checks are the caller's.
int adv_load(ptk_ctx* c, const double* X, int64_t Np, const void* rhs_hist, int hl, int K, hipStream_t s) {
  auto& st = c->adv;
  st.valid = false;
  const int64_t N = c->geom.N;
  const BinGeom bg = bin_geom(c);
  const int64_t n_bins = n_bins_of(bg);
  const int vb = vel_bytes(c);
  const bool vf64 = vb == 8;
  const size_t v3 = (size_t)Np * 3 * vb;
  PTK_TRY(ensure_binning(c, Np, n_bins));
  PTK_TRY(ensure_rebin(c, Np, n_bins));
  PTK_TRY(ensure(c, c->xs, (size_t)Np * 24));
  PTK_TRY(ensure(c, c->xn, (size_t)Np * 24));
  PTK_TRY(ensure(c, c->orig, (size_t)Np * 4));
  PTK_TRY(ensure(c, c->orig_b, (size_t)Np * 4));
  PTK_TRY(ensure(c, c->k1, v3));
  for (int j = 0; j < K; ++j) {
    PTK_TRY(ensure(c, c->abh[j], v3));
    PTK_TRY(ensure(c, c->abh_b[j], v3));
  }
  PTK_TRY(check_binning_caps(c, Np, n_bins));
  PTK_TRY(check_rebin_caps(c, Np, n_bins));
  PTK_TRY(need(c, c->xs, (size_t)Np * 24, "positions"));
  PTK_TRY(need(c, c->xn, (size_t)Np * 24, "positions"));
  PTK_TRY(need(c, c->orig, (size_t)Np * 4, "caller index"));
  PTK_TRY(need(c, c->orig_b, (size_t)Np * 4, "caller index"));
  PTK_TRY(need(c, c->k1, v3, "velocities"));
  for (int j = 0; j < K; ++j) {
    PTK_TRY(need(c, c->abh[j], v3, "history"));
    PTK_TRY(need(c, c->abh_b[j], v3, "history"));
  }
  c->bin_valid = false;  // the sort below reuses the interpolate calls' sort buffers
  uint32_t* keys = (uint32_t*)c->keys_a.ptr;
  int* flag = (int*)c->flag.ptr;
  PTK_HIP(c, launch_fill_i32(flag, 1, 0, s), "flag clear");
  if (Np > 0) {
    {
      Timed t(c, s, PTK_T_KEYS);
      PTK_HIP(c, launch_keys(X, Np, (int)N, invd_of(N), bg, keys, flag, s), "keys");
    }
    uint32_t* perm = nullptr;
    {
      Timed t(c, s, PTK_T_SORT);
      uint32_t* sk = nullptr;
      PTK_TRY(bin_sorted(c, Np, n_bins, &perm, s, &sk, (uint32_t*)c->aoff.ptr));
      PTK_HIP(c, hipMemcpyAsync(c->skeys.ptr, sk, (size_t)Np * 4, hipMemcpyDeviceToDevice, s), "sorted keys");
    }
    Timed t(c, s, PTK_T_PERMUTE);
    PTK_HIP(c, gather3_f64(X, perm, Np, (double*)c->xs.ptr, s), "gather positions");
    PTK_HIP(c, hipMemcpyAsync(c->orig.ptr, perm, (size_t)Np * 4, hipMemcpyDeviceToDevice, s), "copy order");
    for (int j = 0; j < hl; ++j) {
      const char* in = (const char*)rhs_hist + j * v3;
      PTK_HIP(c,
              vf64 ? gather3_f64((const double*)in, perm, Np, (double*)c->abh[j].ptr, s)
                   : gather3_f32((const float*)in, perm, Np, (float*)c->abh[j].ptr, s),
              "gather history");
    }
  }
  st.ori = false;
  st.inert = false;
  st.Np = Np;
  st.N = N;
  st.vb = vb;
  st.K = K;
  st.hl = K ? hl : 0;
  st.xcur = (double*)c->xs.ptr;
  st.xnext = (double*)c->xn.ptr;
  st.xrow = nullptr;
  st.orig = (uint32_t*)c->orig.ptr;
  st.orig_b = (uint32_t*)c->orig_b.ptr;
  st.k1 = c->k1.ptr;
  for (int j = 0; j < 4; ++j) {
    st.h[j] = j < K ? c->abh[j].ptr : nullptr;
    st.hb[j] = j < K ? c->abh_b[j].ptr : nullptr;
  }
  st.valid = true;
  return PTK_OK;
}

// nsteps steps of the loaded state on the current field.  With final_X (the
// one-shot form) the last step writes the positions, and the history to
// final_hist, straight to the caller's order and skips its re-binning, which
// leaves no loaded state; otherwise every step re-bins and the state stays
// loaded.  grad_out: the last step's velocity gradient, caller order.
int adv_steps(ptk_ctx* c, int scheme, double dt, int nsteps, void* grad_out, hipStream_t s, double* final_X,
              void* final_hist, bool stage2_next = false) {
  auto& st = c->adv;
  const int64_t Np = st.Np;
  const int64_t N = c->geom.N;
  const BinGeom bg = bin_geom(c);
  const int64_t n_bins = n_bins_of(bg);
  const double invd = invd_of(N);
  const int vb = vel_bytes(c);
  const bool vf64 = vb == 8;
  const size_t v3 = (size_t)Np * 3 * vb;
  const int K = ab_order(scheme);
  if (st.K == 0) {
    // no history: the velocity buffer may change width with the storage type
    PTK_TRY(ensure(c, c->k1, v3));
    st.k1 = c->k1.ptr;
  }
  if (scheme == PTK_HEUN) PTK_TRY(ensure(c, c->k2, v3));
  const bool ori = st.ori, inert = st.inert;
  const bool pst = ori || inert;  // a per-particle 3-vector state beside X (axes or velocities)
  const size_t g9 = (size_t)Np * 9 * vb, p3 = (size_t)Np * 24;
  if (ori) PTK_TRY(ensure(c, c->gint, g9));
  if (pst) {
    // the stage rhs and the predictor's axes (velocities) and gradient (the
    // state and its history were allocated when it was set)
    PTK_TRY(ensure(c, c->ori_r1, p3));
    PTK_TRY(ensure(c, c->ori_r2, p3));
    PTK_TRY(ensure(c, c->ori_ps, p3));
    if (scheme == PTK_HEUN && ori) PTK_TRY(ensure(c, c->gint2, g9));
    if (st.K == 0) st.r1 = (double*)c->ori_r1.ptr;
    st.r2 = (double*)c->ori_r2.ptr;
    st.ps = (double*)c->ori_ps.ptr;
  }
  // every buffer the steps below write, by its capacity (the state's
  // pointers rotate among these buffers)
  PTK_TRY(check_binning_caps(c, Np, n_bins));
  PTK_TRY(check_rebin_caps(c, Np, n_bins));
  {
    const DevBuf* pos[] = {&c->xs, &c->xn};
    for (const DevBuf* b : pos) PTK_TRY(need(c, *b, (size_t)Np * 24, "positions"));
    const DevBuf* idx[] = {&c->orig, &c->orig_b};
    for (const DevBuf* b : idx) PTK_TRY(need(c, *b, (size_t)Np * 4, "caller index"));
    PTK_TRY(need(c, c->k1, v3, "velocities"));
    for (int j = 0; j < st.K; ++j) {
      PTK_TRY(need(c, c->abh[j], v3, "history"));
      PTK_TRY(need(c, c->abh_b[j], v3, "history"));
    }
    if (scheme == PTK_HEUN) PTK_TRY(need(c, c->k2, v3, "predictor velocities"));
    if (ori) PTK_TRY(need(c, c->gint, g9, "gradients"));
    if (pst) {
      const DevBuf* o3[] = {&c->ori_p, &c->ori_pn, &c->ori_r1, &c->ori_r2, &c->ori_ps};
      for (const DevBuf* b : o3) PTK_TRY(need(c, *b, p3, "per-particle state"));
      for (int j = 0; j < st.K; ++j) {
        PTK_TRY(need(c, c->ori_h[j], p3, "per-particle state history"));
        PTK_TRY(need(c, c->ori_hb[j], p3, "per-particle state history"));
        if (inert) {
          PTK_TRY(need(c, c->in_vh[j], p3, "velocity history"));
          PTK_TRY(need(c, c->in_vhb[j], p3, "velocity history"));
        }
      }
      if (scheme == PTK_HEUN && ori) PTK_TRY(need(c, c->gint2, g9, "predictor gradients"));
    }
  }

  uint32_t* keys = (uint32_t*)c->keys_a.ptr;
  int* flag = (int*)c->flag.ptr;
  void* k2 = c->k2.ptr;
  int hl = st.hl;
  auto gather_v = [&](const void* in, const uint32_t* pm, void* out) -> hipError_t {
    return vf64 ? gather3_f64((const double*)in, pm, Np, (double*)out, s)
                : gather3_f32((const float*)in, pm, Np, (float*)out, s);
  };
  auto scatter_v = [&](const void* in, const uint32_t* idx, int width, void* out) -> hipError_t {
    return vf64 ? scatter_f64((const double*)in, idx, Np, width, (double*)out, s)
                : scatter_f32((const float*)in, idx, Np, width, (float*)out, s);
  };
  // Positions: particle i of the current bin order is row xrow[i] of xcur
  // (row i while xrow is NULL); every update writes its result in the current
  // bin order to xnext.  After a re-binning the next step reads xnext through
  // the new permutation instead of gathering it: the permutation of one time
  // step is close to the identity, so those reads stay nearly unit-stride.
  // (inertial particles move with their own FP64 velocities)
  auto update = [&](int kind, const UpdateVel& v) -> int {
    Timed t(c, s, PTK_T_UPDATE);
    PTK_HIP(c,
            launch_update(kind, inert ? 1 : vf64, st.xcur, st.xrow, v, dt, Np, st.xnext, keys, (int)N, invd, bg, flag,
                          s),
            "position update");
    return PTK_OK;
  };
  auto vel = [](const void* a, const void* b) {
    UpdateVel v;
    std::memset(&v, 0, sizeof(v));
    v.k[0] = a;
    v.k[1] = b;
    v.nk = b ? 2 : 1;
    return v;
  };
  // re-bin relative to the current (bin-ordered) state: new keys in `keys`;
  // writes the permutation to `out` (aperm after a step, aperm_p for the Heun
  // predictor, so that the step's own permutation, xrow, survives it) and the
  // new sorted keys / offsets to skeys2 / offsets2 (the current ones, skeys /
  // aoff, stay valid until swap_bins)
  auto rebin = [&](uint32_t* out) -> int {
    Timed t(c, s, PTK_T_SORT);
    RebinScratch w;
    w.in_start = (uint32_t*)c->rb_in.ptr;
    w.out_before = (uint32_t*)c->rb_out.ptr;
    w.inc_before = (uint32_t*)c->rb_inc.ptr;
    w.blockoff = (uint32_t*)c->rb_block.ptr;
    w.mk_a = (uint32_t*)c->mk_a.ptr;
    w.mk_b = (uint32_t*)c->mk_b.ptr;
    w.mv_a = (uint32_t*)c->mv_a.ptr;
    w.mv_b = (uint32_t*)c->mv_b.ptr;
    w.mo = (uint32_t*)c->mo.ptr;
    w.hist = (uint32_t*)c->hist.ptr;
    w.scan_tmp = (uint32_t*)c->scan_tmp.ptr;
    PTK_HIP(c,
            rebin_incremental((const uint32_t*)c->skeys.ptr, (const uint32_t*)c->aoff.ptr, keys, Np, n_bins,
                              bits_for(n_bins), w, out, (uint32_t*)c->skeys2.ptr, (uint32_t*)c->offsets2.ptr, s),
            "re-bin");
    return PTK_OK;
  };
  auto swap_bins = [&]() {
    std::swap(c->skeys, c->skeys2);
    std::swap(c->aoff, c->offsets2);
  };

  PTK_HIP(c, launch_fill_i32(flag, 1, 0, s), "flag clear");
  for (int step = 0; step < nsteps; ++step) {
    const bool last = step == nsteps - 1;
    void* k1 = st.k1;
    // u(X_n), and its gradient, at the bin-ordered positions
    {
      // the last step writes the gradient straight to the caller's order
      InterpArgs a = base_args(c);
      a.offsets = (const uint32_t*)c->aoff.ptr;
      a.X = st.xcur;
      a.xrow = st.xrow;
      a.np = Np;
      a.out = k1;
      // the axes' rhs needs the gradient in bin order at every step; without
      // axes only the last step evaluates it, straight into the caller's order
      a.grad = ori ? c->gint.ptr : grad_out && last ? grad_out : nullptr;
      a.grad_orig = !ori && grad_out && last ? st.orig : nullptr;
      a.out_f64 = vf64;
      {
        Timed t(c, s, a.grad ? PTK_T_INTERP_GRAD : PTK_T_INTERP);
        PTK_HIP(c, launch_interp(c->storage, c->I, a, s), "interpolate");
      }
      if (ori) {
        Timed t(c, s, PTK_T_UPDATE);
        if (grad_out && last) PTK_HIP(c, scatter_v(c->gint.ptr, st.orig, 9, grad_out), "scatter gradient");
        PTK_HIP(c, launch_jeffery_rhs(vf64, c->gint.ptr, st.p, st.shape, Np, st.r1, s), "axis rhs");
      } else if (inert) {
        Timed t(c, s, PTK_T_UPDATE);
        PTK_HIP(c, launch_drag_rhs(vf64, k1, st.p, st.tau, Np, st.r1, s), "drag");
      }
    }
    // the axes' (inertial particles' velocities') update with the stage rhs
    // in v; axes are brought to unit length at the step's end
    auto orient = [&](int kind, const UpdateVel& v, double* out, int unit) -> int {
      Timed t(c, s, PTK_T_UPDATE);
      PTK_HIP(c, launch_orient_update(kind, st.p, v, dt, Np, unit, out, s), "axis update");
      return PTK_OK;
    };
    // axes are normalized at the end of each step, velocities not
    const int unit = ori ? 1 : 0;
    if (scheme == PTK_EULER) {
      PTK_TRY(update(kEulerOrPredict, inert ? vel(st.p, nullptr) : vel(k1, nullptr)));
      if (pst) PTK_TRY(orient(kEulerOrPredict, vel(st.r1, nullptr), st.pn, unit));
    } else if (scheme == PTK_HEUN) {
      // predictor (into xnext), re-binned; u at the predictor is written
      // back in the step's bin order
      PTK_TRY(update(kEulerOrPredict, inert ? vel(st.p, nullptr) : vel(k1, nullptr)));
      if (pst) PTK_TRY(orient(kEulerOrPredict, vel(st.r1, nullptr), st.ps, 0));
      uint32_t* pp = (uint32_t*)c->aperm_p.ptr;
      PTK_TRY(rebin(pp));
      {
        // the kernel reads the predictor positions through pp, the order it
        // also writes u in: no gathered copy.  With stage2_next the second
        // stage sees the field of the step's end time.
        InterpArgs b = base_args(c, stage2_next);
        b.offsets = (const uint32_t*)c->offsets2.ptr;  // the predictor's bins
        b.X = st.xnext;
        b.xrow = pp;
        b.np = Np;
        b.orig = pp;
        b.out = k2;
        b.grad = ori ? c->gint2.ptr : nullptr;  // the axes' second stage needs the gradient there
        b.out_f64 = vf64;
        Timed t(c, s, ori ? PTK_T_INTERP_GRAD : PTK_T_INTERP);
        PTK_HIP(c, launch_interp(c->storage, c->I, b, s), "interpolate predictor");
      }
      PTK_TRY(update(kHeunCorrect, inert ? vel(st.p, st.ps) : vel(k1, k2)));
      if (pst) {
        {
          Timed t(c, s, PTK_T_UPDATE);
          if (ori)
            PTK_HIP(c, launch_jeffery_rhs(vf64, c->gint2.ptr, st.ps, st.shape, Np, st.r2, s), "axis rhs");
          else
            PTK_HIP(c, launch_drag_rhs(vf64, k2, st.ps, st.tau, Np, st.r2, s), "drag");
        }
        PTK_TRY(orient(kHeunCorrect, vel(st.r1, st.r2), st.pn, unit));
      }
    } else {
      // order min(K, hl + 1): u_n = k1 and the hl stored velocities
      const int q = hl + 1 < K ? hl + 1 : K;
      UpdateVel v;
      std::memset(&v, 0, sizeof(v));
      v.k[0] = k1;
      for (int j = 1; j < q; ++j) v.k[j] = st.h[j - 1];
      for (int j = 0; j < q; ++j) v.b[j] = kABW[q][j];
      v.nk = q;
      if (inert) {
        // the positions' history is the earlier particle velocities
        UpdateVel vx = v;
        vx.k[0] = st.p;
        for (int j = 1; j < q; ++j) vx.k[j] = st.vh[j - 1];
        PTK_TRY(update(q == 1 ? kEulerOrPredict : kAB, vx));
      } else {
        PTK_TRY(update(q == 1 ? kEulerOrPredict : kAB, v));
      }
      if (pst) {
        UpdateVel vp = v;
        vp.k[0] = st.r1;
        for (int j = 1; j < q; ++j) vp.k[j] = st.ph[j - 1];
        PTK_TRY(orient(q == 1 ? kEulerOrPredict : kAB, vp, st.pn, unit));
        double* tp = st.ph[K - 1];
        for (int j = K - 1; j > 0; --j) st.ph[j] = st.ph[j - 1];
        st.ph[0] = st.r1;
        st.r1 = tp;
      }
      if (inert) {
        // V_n joins the velocity history; the dropped buffer takes the next
        // step's velocities (gathered into it below)
        double* tv = st.vh[K - 1];
        for (int j = K - 1; j > 0; --j) st.vh[j] = st.vh[j - 1];
        st.vh[0] = st.p;
        st.p = tv;
      }
      // history rotation: u_{n-j-1} <- u_{n-j}, u_n <- k1; the dropped buffer
      // takes the next step's velocity
      void* t = st.h[K - 1];
      for (int j = K - 1; j > 0; --j) st.h[j] = st.h[j - 1];
      st.h[0] = k1;
      st.k1 = t;
      hl = hl < K ? hl + 1 : K;
    }
    if (last && final_X) {
      Timed t(c, s, PTK_T_PERMUTE);
      PTK_HIP(c, scatter_f64(st.xnext, st.orig, Np, 3, final_X, s), "scatter positions");
      for (int j = 0; j < hl; ++j)
        PTK_HIP(c, scatter_v(st.h[j], st.orig, 3, (char*)final_hist + j * v3), "scatter history");
      st.valid = false;
      break;
    }
    // re-bin the new positions and carry the per-particle state along (the
    // positions stay where they are: the next step reads them through perm)
    uint32_t* perm = (uint32_t*)c->aperm.ptr;
    PTK_TRY(rebin(perm));
    {
      Timed t(c, s, PTK_T_PERMUTE);
      PTK_HIP(c, gather_u32(st.orig, perm, Np, st.orig_b, s), "gather order");
      for (int j = 0; j < hl; ++j) PTK_HIP(c, gather_v(st.h[j], perm, st.hb[j]), "gather history");
      if (pst) {
        // the new axes (velocities) into the new bin order (the old ones'
        // buffer takes them)
        PTK_HIP(c, gather3_f64(st.pn, perm, Np, st.p, s), "gather axes");
        for (int j = 0; j < hl; ++j) PTK_HIP(c, gather3_f64(st.ph[j], perm, Np, st.phb[j], s), "gather axis history");
        for (int j = 0; j < hl; ++j) std::swap(st.ph[j], st.phb[j]);
      }
      if (inert) {
        for (int j = 0; j < hl; ++j)
          PTK_HIP(c, gather3_f64(st.vh[j], perm, Np, st.vhb[j], s), "gather velocity history");
        for (int j = 0; j < hl; ++j) std::swap(st.vh[j], st.vhb[j]);
      }
    }
    st.xrow = perm;
    std::swap(st.xcur, st.xnext);
    swap_bins();
    std::swap(st.orig, st.orig_b);
    for (int j = 0; j < hl; ++j) std::swap(st.h[j], st.hb[j]);
  }
  st.hl = hl;
  return check_flag(c, s);
}

// the loaded positions (and history) in the caller's order
int adv_store(ptk_ctx* c, double* X, void* rhs_hist, hipStream_t s) {
  auto& st = c->adv;
  const int64_t Np = st.Np;
  if (Np == 0) return PTK_OK;
  const bool vf64 = st.vb == 8;
  const size_t v3 = (size_t)Np * 3 * st.vb;
  Timed t(c, s, PTK_T_PERMUTE);
  const double* x = st.xcur;
  if (st.xrow) {
    PTK_HIP(c, gather3_f64(st.xcur, st.xrow, Np, st.xnext, s), "gather positions");
    x = st.xnext;
  }
  PTK_HIP(c, scatter_f64(x, st.orig, Np, 3, X, s), "scatter positions");
  for (int j = 0; j < st.hl; ++j) {
    char* out = (char*)rhs_hist + j * v3;
    PTK_HIP(c,
            vf64 ? scatter_f64((const double*)st.h[j], st.orig, Np, 3, (double*)out, s)
                 : scatter_f32((const float*)st.h[j], st.orig, Np, 3, (float*)out, s),
            "scatter history");
  }
  return PTK_OK;
}

}  // namespace

int ptk_advance_particles(ptk_ctx* c, double* X, int64_t Np, void* rhs_hist, int* hist_len, int scheme,
                          double dt, int nsteps, void* grad_out, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (scheme < PTK_EULER || scheme > PTK_AB4) return fail(c, PTK_EINVAL, "bad scheme");
  // Adams-Bashforth order and history depth
  const int K = ab_order(scheme);
  if (Np < 0 || Np > (int64_t)0xFFFFFFFF) return fail(c, PTK_EINVAL, "Np out of range [0, 2^32)");
  if (nsteps < 0) return fail(c, PTK_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(c, PTK_EINVAL, "dt must be finite");
  if (K) {
    if (!rhs_hist || !hist_len) return fail(c, PTK_EINVAL, "Adams-Bashforth needs rhs_hist and hist_len");
    if (*hist_len < 0 || *hist_len > K) return fail(c, PTK_EINVAL, "hist_len must be in [0, order]");
  }
  if (Np > 0 && !X) return fail(c, PTK_EINVAL, "NULL positions");
  if (Np == 0 || nsteps == 0) return PTK_OK;
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  // the one-shot form runs on the buffers of the loaded state
  c->adv.valid = false;
  PTK_TRY(adv_load(c, X, Np, rhs_hist, K ? *hist_len : 0, K, s));
  const int r = adv_steps(c, scheme, dt, nsteps, grad_out, s, X, rhs_hist);
  if (K && r == PTK_OK) *hist_len = c->adv.hl;
  c->adv.valid = false;
  return r;
}

int ptk_particles_load(ptk_ctx* c, const double* X, int64_t Np, const void* rhs_hist, int hist_len, int hist_depth,
                       void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (Np < 0 || Np > (int64_t)0xFFFFFFFF) return fail(c, PTK_EINVAL, "Np out of range [0, 2^32)");
  if (Np > 0 && !X) return fail(c, PTK_EINVAL, "NULL positions");
  if (hist_depth < 0 || hist_depth > 4 || hist_depth == 1)
    return fail(c, PTK_EINVAL, "hist_depth must be 0 or an Adams-Bashforth order 2..4");
  if (hist_len < 0 || hist_len > hist_depth) return fail(c, PTK_EINVAL, "hist_len must be in [0, hist_depth]");
  if (hist_len > 0 && Np > 0 && !rhs_hist) return fail(c, PTK_EINVAL, "NULL history");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  PTK_TRY(adv_load(c, X, Np, rhs_hist, hist_len, hist_depth, s));
  const int r = check_flag(c, s);
  if (r != PTK_OK) c->adv.valid = false;
  return r;
}

int ptk_particles_advance(ptk_ctx* c, int scheme, double dt, int nsteps, void* grad_out, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->adv.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (scheme < PTK_EULER || scheme > PTK_AB4) return fail(c, PTK_EINVAL, "bad scheme");
  if (nsteps < 0) return fail(c, PTK_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(c, PTK_EINVAL, "dt must be finite");
  if (c->geom.N != c->adv.N) return fail(c, PTK_EINVAL, "the field's grid differs from the loaded particles' bins");
  const int K = ab_order(scheme);
  if (K && K != c->adv.K) return fail(c, PTK_EINVAL, "Adams-Bashforth order differs from the loaded history depth");
  if (c->adv.K && vel_bytes(c) != c->adv.vb)
    return fail(c, PTK_EINVAL, "the storage type changes the loaded history's precision");
  if (c->adv.Np == 0 || nsteps == 0) return PTK_OK;
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  return adv_steps(c, scheme, dt, nsteps, grad_out, S(stream), nullptr, nullptr);
}

int ptk_particles_set_orientation(ptk_ctx* c, const double* p, const double* p_hist, int hist_len, double shape,
                                  void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  auto& st = c->adv;
  if (!st.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  if (!(shape >= -1.0 && shape <= 1.0)) return fail(c, PTK_EINVAL, "shape must be in [-1, 1]");
  if (st.Np > 0 && !p) return fail(c, PTK_EINVAL, "NULL axes");
  if (hist_len != (st.K ? st.hl : 0))
    return fail(c, PTK_EINVAL, "hist_len must equal the loaded position history's length");
  if (hist_len > 0 && st.Np > 0 && !p_hist) return fail(c, PTK_EINVAL, "NULL axis history");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int64_t Np = st.Np;
  const size_t p3 = (size_t)Np * 24;
  st.ori = false;
  st.inert = false;  // axes replace inertia (they share the state slots)
  PTK_TRY(ensure(c, c->ori_p, p3));
  PTK_TRY(ensure(c, c->ori_pn, p3));
  PTK_TRY(ensure(c, c->ori_r1, p3));
  for (int j = 0; j < st.K; ++j) {
    PTK_TRY(ensure(c, c->ori_h[j], p3));
    PTK_TRY(ensure(c, c->ori_hb[j], p3));
  }
  PTK_TRY(need(c, c->ori_p, p3, "axes"));
  st.p = (double*)c->ori_p.ptr;
  st.pn = (double*)c->ori_pn.ptr;
  st.r1 = (double*)c->ori_r1.ptr;
  for (int j = 0; j < 4; ++j) {
    st.ph[j] = j < st.K ? (double*)c->ori_h[j].ptr : nullptr;
    st.phb[j] = j < st.K ? (double*)c->ori_hb[j].ptr : nullptr;
  }
  if (Np > 0) {
    // into the current bin order: particle i is the caller's orig[i]
    PTK_HIP(c, gather3_f64(p, st.orig, Np, st.p, s), "gather axes");
    for (int j = 0; j < hist_len; ++j)
      PTK_HIP(c, gather3_f64(p_hist + (size_t)j * Np * 3, st.orig, Np, st.ph[j], s), "gather axis history");
  }
  st.shape = shape;
  st.ori = true;
  return PTK_OK;
}

int ptk_particles_get_orientation(ptk_ctx* c, double* p, double* p_hist, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  auto& st = c->adv;
  if (!st.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  if (!st.ori) return fail(c, PTK_EINVAL, "the loaded particles carry no axes");
  const int hl = st.K ? st.hl : 0;
  if (st.Np > 0 && (!p || (hl > 0 && !p_hist))) return fail(c, PTK_EINVAL, "NULL pointer");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int64_t Np = st.Np;
  if (Np == 0) return PTK_OK;
  PTK_HIP(c, scatter_f64(st.p, st.orig, Np, 3, p, s), "scatter axes");
  for (int j = 0; j < hl; ++j)
    PTK_HIP(c, scatter_f64(st.ph[j], st.orig, Np, 3, p_hist + (size_t)j * Np * 3, s), "scatter axis history");
  return PTK_OK;
}

int ptk_particles_set_inertia(ptk_ctx* c, const double* V, const double* v_hist, const double* r_hist, int hist_len,
                              double tau, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  auto& st = c->adv;
  if (!st.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(c, PTK_EINVAL, "tau must be positive and finite");
  if (st.Np > 0 && !V) return fail(c, PTK_EINVAL, "NULL velocities");
  if (hist_len != (st.K ? st.hl : 0))
    return fail(c, PTK_EINVAL, "hist_len must equal the loaded position history's length");
  if (hist_len > 0 && st.Np > 0 && (!v_hist || !r_hist)) return fail(c, PTK_EINVAL, "NULL history");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int64_t Np = st.Np;
  const size_t p3 = (size_t)Np * 24;
  st.ori = false;  // inertia replaces axes (they share the state slots)
  st.inert = false;
  PTK_TRY(ensure(c, c->ori_p, p3));
  PTK_TRY(ensure(c, c->ori_pn, p3));
  PTK_TRY(ensure(c, c->ori_r1, p3));
  for (int j = 0; j < st.K; ++j) {
    PTK_TRY(ensure(c, c->ori_h[j], p3));
    PTK_TRY(ensure(c, c->ori_hb[j], p3));
    PTK_TRY(ensure(c, c->in_vh[j], p3));
    PTK_TRY(ensure(c, c->in_vhb[j], p3));
  }
  PTK_TRY(need(c, c->ori_p, p3, "velocities"));
  st.p = (double*)c->ori_p.ptr;
  st.pn = (double*)c->ori_pn.ptr;
  st.r1 = (double*)c->ori_r1.ptr;
  for (int j = 0; j < 4; ++j) {
    st.ph[j] = j < st.K ? (double*)c->ori_h[j].ptr : nullptr;
    st.phb[j] = j < st.K ? (double*)c->ori_hb[j].ptr : nullptr;
    st.vh[j] = j < st.K ? (double*)c->in_vh[j].ptr : nullptr;
    st.vhb[j] = j < st.K ? (double*)c->in_vhb[j].ptr : nullptr;
  }
  if (Np > 0) {
    // into the current bin order: particle i is the caller's orig[i]
    PTK_HIP(c, gather3_f64(V, st.orig, Np, st.p, s), "gather velocities");
    for (int j = 0; j < hist_len; ++j) {
      PTK_HIP(c, gather3_f64(v_hist + (size_t)j * Np * 3, st.orig, Np, st.vh[j], s), "gather velocity history");
      PTK_HIP(c, gather3_f64(r_hist + (size_t)j * Np * 3, st.orig, Np, st.ph[j], s), "gather drag history");
    }
  }
  st.tau = tau;
  st.inert = true;
  return PTK_OK;
}

int ptk_particles_get_inertia(ptk_ctx* c, double* V, double* v_hist, double* r_hist, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  auto& st = c->adv;
  if (!st.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  if (!st.inert) return fail(c, PTK_EINVAL, "the loaded particles carry no inertia");
  const int hl = st.K ? st.hl : 0;
  if (st.Np > 0 && (!V || (hl > 0 && (!v_hist || !r_hist)))) return fail(c, PTK_EINVAL, "NULL pointer");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int64_t Np = st.Np;
  if (Np == 0) return PTK_OK;
  PTK_HIP(c, scatter_f64(st.p, st.orig, Np, 3, V, s), "scatter velocities");
  for (int j = 0; j < hl; ++j) {
    PTK_HIP(c, scatter_f64(st.vh[j], st.orig, Np, 3, v_hist + (size_t)j * Np * 3, s), "scatter velocity history");
    PTK_HIP(c, scatter_f64(st.ph[j], st.orig, Np, 3, r_hist + (size_t)j * Np * 3, s), "scatter drag history");
  }
  return PTK_OK;
}

namespace {

// ---- particle state files (in the caller's order, Sec. 3.4)
struct StateHeader {
  char magic[8];       // "PTKSTATE"
  uint32_t version;    // 1
  uint32_t flags;      // bit 0: axes (and their history) follow; bit 1: inertia (V and its histories)
  int64_t np;
  int32_t depth;       // Adams-Bashforth history depth k (0 without history)
  int32_t hist_len;    // valid history entries
  int32_t vel_bytes;   // 8 (FP64 storage) or 4
  int32_t grid;        // N of the field the state was saved with
  double shape;        // axes' shape factor
  uint64_t reserved[2];  // [0]: inertial particles' response time tau (float64 bits)
};
static_assert(sizeof(StateHeader) == 64, "state header is 64 bytes");
constexpr size_t kIoChunk = (size_t)32 << 20;

// Device <-> file copies through one pinned host buffer of kIoChunk bytes.
struct PinnedChunk {
  void* p = nullptr;
  ~PinnedChunk() {
    if (p) (void)hipHostFree(p);
  }
};

int write_device(ptk_ctx* c, FILE* f, const void* dev, size_t bytes, PinnedChunk& h, hipStream_t s) {
  for (size_t off = 0; off < bytes; off += kIoChunk) {
    const size_t n = bytes - off < kIoChunk ? bytes - off : kIoChunk;
    PTK_HIP(c, hipMemcpyAsync(h.p, (const char*)dev + off, n, hipMemcpyDeviceToHost, s), "state copy to host");
    PTK_HIP(c, hipStreamSynchronize(s), "stream synchronize");
    if (fwrite(h.p, 1, n, f) != n) return fail(c, PTK_EIO, "short write of the state file");
  }
  return PTK_OK;
}

int read_device(ptk_ctx* c, FILE* f, void* dev, size_t bytes, PinnedChunk& h, hipStream_t s) {
  for (size_t off = 0; off < bytes; off += kIoChunk) {
    const size_t n = bytes - off < kIoChunk ? bytes - off : kIoChunk;
    if (fread(h.p, 1, n, f) != n) return fail(c, PTK_EIO, "the state file is shorter than its header says");
    PTK_HIP(c, hipMemcpyAsync((char*)dev + off, h.p, n, hipMemcpyHostToDevice, s), "state copy to device");
    PTK_HIP(c, hipStreamSynchronize(s), "stream synchronize");
  }
  return PTK_OK;
}

struct FileCloser {
  FILE* f;
  ~FileCloser() {
    if (f) fclose(f);
  }
};

}  // namespace

int ptk_particles_save(ptk_ctx* c, const char* path, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  auto& st = c->adv;
  if (!path) return fail(c, PTK_EINVAL, "NULL path");
  if (!st.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int64_t Np = st.Np;
  const int hl = st.K ? st.hl : 0;
  const size_t x3 = (size_t)Np * 24, v3 = (size_t)Np * 3 * st.vb;
  // the state in the caller's order, staged on the device (positions, then
  // each history entry, then the axes and theirs, or the velocities and
  // their two histories)
  const size_t total = x3 + (size_t)hl * v3 + (st.ori ? x3 + (size_t)hl * x3 : 0) +
                       (st.inert ? x3 + (size_t)2 * hl * x3 : 0);
  PTK_TRY(ensure(c, c->io, total > 0 ? total : 256));
  PTK_TRY(need(c, c->io, total, "state staging"));
  char* dst = (char*)c->io.ptr;
  if (Np > 0) {
    PTK_TRY(adv_store(c, (double*)dst, dst + x3, s));
    if (st.ori)
      PTK_TRY(ptk_particles_get_orientation(c, (double*)(dst + x3 + (size_t)hl * v3),
                                            (double*)(dst + x3 + (size_t)hl * v3 + x3), stream));
    if (st.inert) {
      char* b = dst + x3 + (size_t)hl * v3;
      PTK_TRY(ptk_particles_get_inertia(c, (double*)b, (double*)(b + x3), (double*)(b + x3 + (size_t)hl * x3), stream));
    }
  }
  StateHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, "PTKSTATE", 8);
  hd.version = 1;
  hd.flags = (st.ori ? 1u : 0u) | (st.inert ? 2u : 0u);
  hd.np = Np;
  hd.depth = st.K;
  hd.hist_len = hl;
  hd.vel_bytes = st.vb;
  hd.grid = (int32_t)st.N;
  hd.shape = st.ori ? st.shape : 0.0;
  if (st.inert) std::memcpy(&hd.reserved[0], &st.tau, sizeof(double));
  FileCloser fc{fopen(path, "wb")};
  if (!fc.f) return fail(c, PTK_EIO, std::string("cannot open ") + path + " for writing");
  if (fwrite(&hd, sizeof(hd), 1, fc.f) != 1) return fail(c, PTK_EIO, "short write of the state header");
  PinnedChunk h;
  PTK_HIP(c, hipHostMalloc(&h.p, kIoChunk, hipHostMallocDefault), "pinned host buffer");
  PTK_TRY(write_device(c, fc.f, dst, total, h, s));
  if (fflush(fc.f) != 0) return fail(c, PTK_EIO, "flush of the state file failed");
  return PTK_OK;
}

int ptk_particles_restore(ptk_ctx* c, const char* path, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!path) return fail(c, PTK_EINVAL, "NULL path");
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  FileCloser fc{fopen(path, "rb")};
  if (!fc.f) return fail(c, PTK_EIO, std::string("cannot open ") + path);
  StateHeader hd;
  if (fread(&hd, sizeof(hd), 1, fc.f) != 1 || std::memcmp(hd.magic, "PTKSTATE", 8) != 0 || hd.version != 1)
    return fail(c, PTK_EIO, "not a particle state file of this version");
  if (hd.np < 0 || hd.np > (int64_t)0xFFFFFFFF || !(hd.depth == 0 || (hd.depth >= 2 && hd.depth <= 4)) ||
      hd.hist_len < 0 || hd.hist_len > hd.depth || (hd.vel_bytes != 4 && hd.vel_bytes != 8) ||
      (hd.flags & ~3u) != 0 || hd.flags == 3u || !(hd.shape >= -1.0 && hd.shape <= 1.0))
    return fail(c, PTK_EIO, "corrupt particle state header");
  double tau = 0.0;
  std::memcpy(&tau, &hd.reserved[0], sizeof(double));
  if ((hd.flags & 2u) && !(tau > 0.0 && std::isfinite(tau))) return fail(c, PTK_EIO, "corrupt particle state header");
  if (hd.grid != (int32_t)c->geom.N) return fail(c, PTK_EINVAL, "the state was saved on a grid of another N");
  if (hd.depth > 0 && hd.vel_bytes != vel_bytes(c))
    return fail(c, PTK_EINVAL, "the state's history has another velocity precision than the field's storage");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int64_t Np = hd.np;
  const int hl = hd.hist_len;
  const bool axes = hd.flags & 1u, inertia = hd.flags & 2u;
  const size_t x3 = (size_t)Np * 24, v3 = (size_t)Np * 3 * hd.vel_bytes;
  const size_t total = x3 + (size_t)hl * v3 + (axes ? x3 + (size_t)hl * x3 : 0) +
                       (inertia ? x3 + (size_t)2 * hl * x3 : 0);
  PTK_TRY(ensure(c, c->io, total > 0 ? total : 256));
  PTK_TRY(need(c, c->io, total, "state staging"));
  char* src = (char*)c->io.ptr;
  PinnedChunk h;
  PTK_HIP(c, hipHostMalloc(&h.p, kIoChunk, hipHostMallocDefault), "pinned host buffer");
  PTK_TRY(read_device(c, fc.f, src, total, h, s));
  c->adv.valid = false;
  PTK_TRY(adv_load(c, (const double*)src, Np, src + x3, hl, hd.depth, s));
  PTK_TRY(check_flag(c, s));
  if (axes)
    PTK_TRY(ptk_particles_set_orientation(c, (const double*)(src + x3 + (size_t)hl * v3),
                                          (const double*)(src + x3 + (size_t)hl * v3 + x3), hl, hd.shape, stream));
  if (inertia) {
    const char* b = src + x3 + (size_t)hl * v3;
    PTK_TRY(ptk_particles_set_inertia(c, (const double*)b, (const double*)(b + x3),
                                      (const double*)(b + x3 + (size_t)hl * x3), hl, tau, stream));
  }
  return PTK_OK;
}

int ptk_particles_step_next_field(ptk_ctx* c, double dt, void* grad_out, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->adv.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  if (!c->has_field) return fail(c, PTK_ENOFIELD, "no field set");
  if (!c->has_next) return fail(c, PTK_ENOFIELD, "no next field: set it with ptk_set_field_next");
  if (!std::isfinite(dt)) return fail(c, PTK_EINVAL, "dt must be finite");
  if (c->geom.N != c->adv.N) return fail(c, PTK_EINVAL, "the field's grid differs from the loaded particles' bins");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  if (c->adv.Np > 0) PTK_TRY(adv_steps(c, PTK_HEUN, dt, 1, grad_out, S(stream), nullptr, nullptr, true));
  // the end time's field is now the current one; the old current buffer is
  // kept for the next call of ptk_set_field_next
  std::swap(c->field, c->field_next);
  std::swap(c->geom, c->geom_next);
  std::swap(c->scale, c->scale_next);
  c->has_next = false;
  c->bin_valid = false;
  return PTK_OK;
}

int ptk_particles_store(ptk_ctx* c, double* X, void* rhs_hist, int* hist_len, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!c->adv.valid) return fail(c, PTK_EINVAL, "no particles loaded");
  if (c->adv.Np > 0 && !X) return fail(c, PTK_EINVAL, "NULL positions");
  if (c->adv.K && (!hist_len || (c->adv.hl > 0 && !rhs_hist)))
    return fail(c, PTK_EINVAL, "the loaded history needs rhs_hist and hist_len");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  PTK_TRY(adv_store(c, X, rhs_hist, S(stream)));
  if (hist_len) *hist_len = c->adv.K ? c->adv.hl : 0;
  return PTK_OK;
}

int ptk_timing_enable(ptk_ctx* c, int enable) {
  if (!c) return PTK_EINVAL;
  DeviceGuard g(c->device);
  drain_timers(c);
  for (int k = 0; k < kTimerKinds; ++k) {
    c->timer_ms[k] = 0.0;
    c->timer_count[k] = 0;
  }
  c->timing = enable != 0;
  return PTK_OK;
}

int ptk_timing_read(ptk_ctx* c, double* ms, int64_t* launches) {
  if (!c) return PTK_EINVAL;
  DeviceGuard g(c->device);
  drain_timers(c);
  for (int k = 0; k < kTimerKinds; ++k) {
    if (ms) ms[k] = c->timer_ms[k];
    if (launches) launches[k] = c->timer_count[k];
  }
  return PTK_OK;
}

int ptk_learned_make_pairs(ptk_ctx* c, const double* X, int64_t Np, uint16_t* feat, float* target,
                           void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  LearnedField lf;
  PTK_TRY(learned_field(c, &lf));
  if (Np < 0 || Np > (int64_t)0xFFFFFFFF) return fail(c, PTK_EINVAL, "Np out of range [0, 2^32)");
  if (Np > 0 && !X) return fail(c, PTK_EINVAL, "NULL positions");
  if (feat && ((uintptr_t)feat & 7) != 0) return fail(c, PTK_EINVAL, "feature rows must be 8-byte aligned");
  if (Np == 0 || (!feat && !target)) return PTK_OK;
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  if (target) {
    PTK_TRY(ensure(c, c->lwide, (size_t)Np * 12));
    PTK_TRY(need(c, c->lwide, (size_t)Np * 12, "wide-kernel values"));
    PTK_TRY(interp_common(c, X, Np, c->lwide.ptr, nullptr, PTK_F32, stream));
  }
  PTK_HIP(c, launch_fill_i32((int*)c->flag.ptr, 1, 0, s), "flag clear");
  PTK_HIP(c,
          launch_learned_pairs(lf, X, Np, (const float*)c->lwide.ptr, feat, target, (int*)c->flag.ptr, s),
          "training pairs");
  return check_flag(c, s);
}

int ptk_learned_set_params(ptk_ctx* c, const float* params) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!params) return fail(c, PTK_EINVAL, "NULL parameters");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  const size_t pb = (size_t)kLearnedNParams * 4;
  PTK_TRY(ensure(c, c->lparams, pb));
  PTK_TRY(ensure(c, c->lm, pb));
  PTK_TRY(ensure(c, c->lv, pb));
  PTK_TRY(ensure(c, c->lw1b, 128 * 208 * 2));
  PTK_TRY(ensure(c, c->lw2b, 128 * 128 * 2));
  PTK_TRY(ensure(c, c->lw2bt, 128 * 128 * 2));
  PTK_HIP(c, hipDeviceSynchronize(), "synchronize");
  PTK_HIP(c, hipMemcpy(c->lparams.ptr, params, pb, hipMemcpyHostToDevice), "parameter upload");
  PTK_HIP(c, hipMemset(c->lm.ptr, 0, pb), "moment clear");
  PTK_HIP(c, hipMemset(c->lv.ptr, 0, pb), "moment clear");
  PTK_HIP(c, hipMemset(c->lw1b.ptr, 0, 128 * 208 * 2), "weight clear");
  LearnedUpdate u;
  std::memset(&u, 0, sizeof(u));
  u.mode = 2;
  PTK_HIP(c,
          launch_learned_update((float*)c->lparams.ptr, (float*)c->lm.ptr, (float*)c->lv.ptr, nullptr, nullptr, u,
                                (uint16_t*)c->lw1b.ptr, (uint16_t*)c->lw2b.ptr, (uint16_t*)c->lw2bt.ptr, nullptr),
          "weight copies");
  PTK_HIP(c, hipDeviceSynchronize(), "synchronize");
  c->learned_ready = true;
  c->learned_step = 0;
  return PTK_OK;
}

int ptk_learned_get_params(ptk_ctx* c, float* params) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  if (!params) return fail(c, PTK_EINVAL, "NULL parameters");
  if (!c->learned_ready) return fail(c, PTK_EINVAL, "no network parameters set");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  PTK_HIP(c, hipDeviceSynchronize(), "synchronize");
  PTK_HIP(c, hipMemcpy(params, c->lparams.ptr, (size_t)kLearnedNParams * 4, hipMemcpyDeviceToHost),
          "parameter download");
  return PTK_OK;
}

int ptk_learned_loss_grad(ptk_ctx* c, const uint16_t* feat, const float* target, int64_t n, float* loss,
                          float* grad, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  PTK_TRY(check_rows(c, feat, target, n));
  if (!loss || !grad) return fail(c, PTK_EINVAL, "NULL output");
  if (n < 64 || n > kLearnedMaxBatch || n % 64) return fail(c, PTK_EINVAL, "n must be a multiple of 64 in [64, 16384]");
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  PTK_TRY(ensure_partials(c, n));
  PTK_HIP(c,
          launch_learned_forward_backward(feat, target, n, (const float*)c->lparams.ptr, (const uint16_t*)c->lw1b.ptr,
                                          (const uint16_t*)c->lw2b.ptr, (const uint16_t*)c->lw2bt.ptr,
                                          (float*)c->lgpart.ptr, (float*)c->llpart.ptr, s),
          "forward and backward");
  LearnedUpdate u;
  std::memset(&u, 0, sizeof(u));
  u.mode = 0;
  u.nparts = (int)(n / 64);
  u.loss_scale = (float)(1.0 / (3.0 * (double)n));
  u.loss_out = loss;
  u.grad_out = grad;
  PTK_HIP(c,
          launch_learned_update((float*)c->lparams.ptr, (float*)c->lm.ptr, (float*)c->lv.ptr,
                                (const float*)c->lgpart.ptr, (const float*)c->llpart.ptr, u, (uint16_t*)c->lw1b.ptr,
                                (uint16_t*)c->lw2b.ptr, (uint16_t*)c->lw2bt.ptr, s),
          "gradient sum");
  return PTK_OK;
}

int ptk_learned_train(ptk_ctx* c, const uint16_t* feat, const float* target, int64_t n,
                      const ptk_train_config* cfg, float* loss_curve, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  PTK_TRY(check_rows(c, feat, target, n));
  if (!cfg) return fail(c, PTK_EINVAL, "NULL configuration");
  if (cfg->epochs < 0) return fail(c, PTK_EINVAL, "epochs must be >= 0");
  if (cfg->batch < 64 || cfg->batch > kLearnedMaxBatch || cfg->batch % 64)
    return fail(c, PTK_EINVAL, "batch must be a multiple of 64 in [64, 16384]");
  if (!(cfg->lr > 0.f) || !std::isfinite(cfg->lr)) return fail(c, PTK_EINVAL, "lr must be positive");
  if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f))
    return fail(c, PTK_EINVAL, "betas must be in [0, 1)");
  if (!(cfg->eps > 0.f)) return fail(c, PTK_EINVAL, "eps must be positive");
  if (n < 0) return fail(c, PTK_EINVAL, "n must be >= 0");
  const int64_t nb = n / cfg->batch;
  const int64_t total = (int64_t)cfg->epochs * nb;
  if (total == 0) return PTK_OK;
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  PTK_TRY(ensure_partials(c, cfg->batch));
  const double kPi = 3.14159265358979323846;
  for (int64_t st = 0; st < total; ++st) {
    const int64_t b = st % nb;
    const int64_t r0 = b * cfg->batch;
    const int64_t r1 = ((st + 1) % nb) * cfg->batch;  // the next step's rows
    PTK_HIP(c,
            launch_learned_forward_backward(feat + r0 * kLearnedPitch, target + r0 * 3, cfg->batch,
                                            (const float*)c->lparams.ptr, (const uint16_t*)c->lw1b.ptr,
                                            (const uint16_t*)c->lw2b.ptr, (const uint16_t*)c->lw2bt.ptr,
                                            (float*)c->lgpart.ptr, (float*)c->llpart.ptr, s,
                                            st + 1 < total ? feat + r1 * kLearnedPitch : nullptr),
            "forward and backward");
    const int64_t gs = c->learned_step + 1;
    LearnedUpdate u;
    std::memset(&u, 0, sizeof(u));
    u.mode = 1;
    u.nparts = cfg->batch / 64;
    u.lr = (float)((double)cfg->lr * 0.5 * (1.0 + std::cos(kPi * (double)st / (double)total)));
    u.beta1 = cfg->beta1;
    u.beta2 = cfg->beta2;
    u.eps = cfg->eps;
    u.c1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, (double)gs)));
    u.c2 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta2, (double)gs)));
    u.loss_scale = (float)(1.0 / (3.0 * (double)cfg->batch));
    u.loss_out = loss_curve ? loss_curve + st : nullptr;
    PTK_HIP(c,
            launch_learned_update((float*)c->lparams.ptr, (float*)c->lm.ptr, (float*)c->lv.ptr,
                                  (const float*)c->lgpart.ptr, (const float*)c->llpart.ptr, u,
                                  (uint16_t*)c->lw1b.ptr, (uint16_t*)c->lw2b.ptr, (uint16_t*)c->lw2bt.ptr, s),
            "Adam step");
    c->learned_step = gs;
  }
  return PTK_OK;
}

int ptk_interpolate_learned(ptk_ctx* c, const double* X, int64_t Np, float* out, double audit_frac,
                            double tol_rel_rms, double* audit_rms, int* fell_back, void* stream) {
  if (!c) return PTK_EINVAL;
  c->err.clear();
  LearnedField lf;
  PTK_TRY(learned_field(c, &lf));
  if (!c->learned_ready) return fail(c, PTK_EINVAL, "no network parameters set");
  if (Np < 0 || Np > (int64_t)0xFFFFFFFF) return fail(c, PTK_EINVAL, "Np out of range [0, 2^32)");
  if (!audit_rms || !fell_back) return fail(c, PTK_EINVAL, "NULL audit outputs");
  if (!(audit_frac > 0.0 && audit_frac <= 1.0)) return fail(c, PTK_EINVAL, "audit_frac must be in (0, 1]");
  if (!(tol_rel_rms >= 0.0)) return fail(c, PTK_EINVAL, "tol_rel_rms must be >= 0");
  if (Np > 0 && (!X || !out)) return fail(c, PTK_EINVAL, "NULL pointer");
  *audit_rms = 0.0;
  *fell_back = 0;
  if (Np == 0) return PTK_OK;
  DeviceGuard g(c->device);
  if (g.err != hipSuccess) return hip_fail(c, g.err, "hipSetDevice");
  hipStream_t s = S(stream);
  const int64_t N = c->geom.N;
  const BinGeom bg = bin_geom(c);
  const int64_t n_bins = n_bins_of(bg);
  c->bin_valid = false;
  PTK_TRY(ensure_binning(c, Np, n_bins));
  PTK_HIP(c, launch_fill_i32((int*)c->flag.ptr, 1, 0, s), "flag clear");
  {
    Timed t(c, s, PTK_T_KEYS);
    PTK_HIP(c, launch_keys(X, Np, (int)N, invd_of(N), bg, (uint32_t*)c->keys_a.ptr, (int*)c->flag.ptr, s),
            "keys");
  }
  uint32_t* perm = nullptr;
  {
    Timed t(c, s, PTK_T_SORT);
    PTK_TRY(bin_sorted(c, Np, n_bins, &perm, s));
  }
  {
    // the kernel reads the caller's positions through the permutation
    Timed t(c, s, PTK_T_LEARNED);
    PTK_HIP(c,
            launch_learned_infer(lf, X, Np, perm, (const float*)c->lparams.ptr,
                                 (const uint16_t*)c->lw1b.ptr, (const uint16_t*)c->lw2b.ptr, out, (int*)c->flag.ptr,
                                 s),
            "learned interpolation");
  }
  {
    // positions outside the domain are reported before the audit re-bins
    int h = 0;
    PTK_HIP(c, hipMemcpyAsync(&h, c->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s), "flag read");
    PTK_HIP(c, hipStreamSynchronize(s), "stream synchronize");
    PTK_TRY(flag_error(c, h));
  }
  // audit with the wide kernel at particles 0, k, 2k, ...
  int64_t k = (int64_t)std::llround(1.0 / audit_frac);
  if (k < 1) k = 1;
  const int64_t na = (Np + k - 1) / k;
  PTK_TRY(ensure(c, c->laudit_x, (size_t)na * 24));
  PTK_TRY(ensure(c, c->laudit_u, (size_t)na * 12));
  PTK_TRY(ensure(c, c->laudit_sums, 16));
  PTK_TRY(need(c, c->laudit_x, (size_t)na * 24, "audit positions"));
  PTK_TRY(need(c, c->laudit_u, (size_t)na * 12, "audit values"));
  PTK_TRY(need(c, c->laudit_sums, 16, "audit sums"));
  PTK_HIP(c, launch_stride_gather(X, k, na, (double*)c->laudit_x.ptr, s), "audit positions");
  PTK_TRY(interp_common(c, (const double*)c->laudit_x.ptr, na, c->laudit_u.ptr, nullptr, PTK_F32, stream));
  PTK_HIP(c, launch_audit(out, k, na, (const float*)c->laudit_u.ptr, (double*)c->laudit_sums.ptr, s), "audit");
  double sums[2] = {0.0, 0.0};
  PTK_HIP(c, hipMemcpyAsync(sums, c->laudit_sums.ptr, 16, hipMemcpyDeviceToHost, s), "audit read");
  PTK_HIP(c, hipStreamSynchronize(s), "stream synchronize");
  const double rms = sums[1] > 0.0 ? std::sqrt(sums[0] / sums[1]) : (sums[0] > 0.0 ? INFINITY : 0.0);
  *audit_rms = rms;
  if (!(rms <= tol_rel_rms)) {
    PTK_TRY(interp_common(c, X, Np, out, nullptr, PTK_F32, stream));
    *fell_back = 1;
  }
  return PTK_OK;
}

int ptk_selftest(void) {
  // A context that never touches a device: its buffers hold no allocation
  // (growth is refused by the byte cap before hipMalloc is reached) or a
  // placeholder address that nothing dereferences.
  ptk_ctx c;
  char placeholder[64];
  int bad = 0;
  auto expect = [&](bool ok) { bad += ok ? 0 : 1; };
  // capacity guard: too small, absent, exact, larger
  DevBuf b;
  b.ptr = placeholder;
  b.cap = 1024;
  expect(need(&c, b, 1025, "self-test") == PTK_EINTERNAL && !c.err.empty());
  expect(need(&c, b, 1024, "self-test") == PTK_OK);
  expect(need(&c, b, 16, "self-test") == PTK_OK);
  DevBuf none;
  expect(need(&c, none, 1, "self-test") == PTK_EINTERNAL);
  // growth refused by the byte cap leaves an empty buffer empty and reports
  // PTK_ENOMEM without any runtime call
  c.byte_cap = 4096;
  c.bytes_in_use = 0;
  DevBuf grow;
  expect(ensure(&c, grow, 1 << 20) == PTK_ENOMEM && grow.ptr == nullptr && grow.cap == 0);
  expect(c.bytes_in_use == 0);
  // status bits of the device flag word
  expect(flag_error(&c, 0) == PTK_OK);
  expect(flag_error(&c, kFlagDomain) == PTK_EDOMAIN);
  expect(flag_error(&c, kFlagBinning) == PTK_EINTERNAL);
  expect(flag_error(&c, kFlagDomain | kFlagBinning) == PTK_EDOMAIN);
  // binning and advance buffer checks on a context whose buffers are short
  DevBuf* bufs[] = {&c.keys_a, &c.keys_b, &c.vals_a, &c.vals_b, &c.hist, &c.scan_tmp, &c.offsets};
  for (DevBuf* d : bufs) {
    d->ptr = placeholder;
    d->cap = (size_t)1 << 30;
  }
  expect(check_binning_caps(&c, 1000, 5000) == PTK_OK);
  c.offsets.cap = 4 * 5000;  // one word short of n_bins + 1
  expect(check_binning_caps(&c, 1000, 5000) == PTK_EINTERNAL);
  c.offsets.cap = 4 * 5001;
  c.keys_b.cap = 3999;
  expect(check_binning_caps(&c, 1000, 5000) == PTK_EINTERNAL);
  for (DevBuf* d : bufs) *d = DevBuf();  // nothing for the destructor-free context to release
  return bad == 0 ? PTK_OK : PTK_EINTERNAL;
}

}  // extern "C"
