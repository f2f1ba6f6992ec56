/*
 * ptk.h -- particle-tracking interpolation on one MI355X (gfx950).
 *
 * C ABI of libptk.so.  It computes the particle-tracking hot path of
 * Lalescu, Bramas, Rampp & Wilczek, "An Efficient Particle Tracking Algorithm
 * for Large-Scale Parallel Pseudo-Spectral Simulations of Turbulence":
 * interpolation of a periodic 3-component field given on an N^3 grid at
 * particle positions with I-point tensor-product kernels (Sec. 2.2, the four
 * enumerated steps and Eq. "triple_sum"), its gradient through derivative
 * kernels, and the tracer ODE dX/dt = u(X) (Eq. "tracers") advanced with
 * Euler, Heun or Adams-Bashforth of order 2 to 4 using a per-particle rhs
 * history (Sec. 2.2; Sec. 3.3.1 "Particle data structure").  Beside it: the
 * field set from the solver's spectral state (velocity, or vorticity through
 * the Biot-Savart law of Sec. 2.1; the extra inverse transform of Sec. 4.2),
 * particles kept in the library across steps of a changing field, reduced
 * precision field storage, and a learned correction form.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Domain [0, 2*pi)^3, grid spacing delta = 2*pi/N, node (j1,j2,j3) at
 * j*delta.  Field layout u[x3][x2][x1][a]: x1 fastest, the 3 components
 * fastest within a node (Sec. 2.2 "array of vectorial field values", with the
 * paper's x3-slab convention, Sec. 3.2).  Positions X[p][3] = (x1, x2, x3) in
 * binary64 with |x| < 2^50 (they are reduced modulo 2*pi wherever the field
 * is evaluated; beyond 2^50 the binary64 reduction is no longer exact enough
 * and such positions, like NaN and infinities, are reported as PTK_EDOMAIN).  Gradients
 * grad[p][a][b] = d u_a / d x_b.
 *
 * Pointers named as device pointers must be device memory of the context's
 * GPU, owned by the caller, and must not overlap each other.  Work is enqueued
 * on `stream` (a hipStream_t; NULL = the null stream).  Every call returns after
 * enqueueing, except that it waits for its own work when it has to report a
 * device-side condition (positions outside the domain) -- set PTK_NO_CHECK=1 in the
 * environment to skip that check and the wait.  The library keeps device
 * scratch that grows with the largest call and is freed by ptk_destroy; one
 * context must not be used by two host threads at once, and calls on one
 * context must be issued on one stream or ordered by the caller.
 *
 * Errors: every function returns PTK_OK (0) or a negative code and never
 * throws.  Argument errors are detected before any work is enqueued and leave
 * the context unchanged.  ptk_last_error() describes the last error.
 */
#ifndef PTK_H
#define PTK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ptk_ctx ptk_ctx;

/* Element types of fields, outputs and field storage. */
enum { PTK_F64 = 0, PTK_F32 = 1, PTK_BF16 = 2, PTK_F16 = 3 };

/* Kernel families (Sec. 2.2): Lagrange polynomials, or local splines of
 * smoothness m (m = 0 gives the Lagrange kernel). */
enum { PTK_LAGRANGE = 0, PTK_SPLINE = 1 };

/* Time-stepping schemes for ptk_advance_particles. */
enum { PTK_EULER = 1, PTK_HEUN = 2, PTK_AB2 = 3, PTK_AB3 = 4, PTK_AB4 = 5 };

/* Return codes. */
enum {
  PTK_OK = 0,
  PTK_EINVAL = -1,        /* bad argument (NULL pointer, size, enum value) */
  PTK_ENOFIELD = -2,      /* no field set on the context */
  PTK_ENOMEM = -3,        /* device allocation failed (or the test byte cap) */
  PTK_EHIP = -4,          /* a HIP runtime call failed */
  PTK_EDOMAIN = -5,       /* a position was NaN, infinite or |x| >= 2^50 */
  PTK_EUNSUPPORTED = -6,  /* valid but unsupported request (e.g. odd I) */
  PTK_EIO = -8,           /* a state file could not be written or read, or is
                             not a state file of this version */
  PTK_EINTERNAL = -7      /* an internal consistency check failed (a scratch
                             buffer smaller than a launch needs, or a particle
                             outside the tile its bin names); nothing was
                             written out of bounds */
};

/* Interpolation kernel: family, points per direction I (even; 4, 6 or 8 here)
 * and smoothness m (0 <= m <= I/2 - 1; ignored for PTK_LAGRANGE).  Nodes of a
 * particle in cell c are c + i, i = 1 - I/2 .. I/2 per axis (Eq. "triple_sum").
 * Spline (I = 2n+2, m): on each cell the degree-(2n+1) polynomial that takes the
 * node values at the cell ends, takes at each end the derivatives 1..m of the
 * centred degree-2n Lagrange interpolant about that end, and interpolates the
 * 2(n-m) nodes nearest the cell. */
typedef struct {
  int family;
  int I;
  int m;
} ptk_kernel;

/* Coefficients of the kernel polynomials as the library derives them (exact
 * rationals rounded once to binary64): val[j*I + p] is the coefficient of t^p
 * of beta for node offset j - (I/2 - 1), der[j*I + p] that of d beta/dt (its
 * last column is 0).  Host buffers of I*I doubles each; der may be NULL.
 * Host-only, needs no device or context. */
int ptk_kernel_table(const ptk_kernel *k, double *val, double *der);

/* The same polynomials in powers of (t - 1/2), the form the kernels evaluate
 * (by Horner's rule at t - 1/2, which on [0, 1) loses far less to
 * cancellation than powers of t): val[j*I + p] is the coefficient of
 * (t - 1/2)^p of beta for node offset j - (I/2 - 1), der[j*I + p] that of
 * d beta/dt; each exact rational rounded once (to nearest even) to binary64
 * (val, der) and to binary32 (val32, der32).  Host buffers of I*I elements;
 * der, val32 and der32 may be NULL.  Host-only. */
int ptk_kernel_table_centred(const ptk_kernel *k, double *val, double *der, float *val32, float *der32);

/* Create a context on HIP device `device`.  *out receives the handle. */
int ptk_create(ptk_ctx **out, int device);

/* Release the context, its field copy and its scratch.  NULL is accepted. */
void ptk_destroy(ptk_ctx *ctx);

/* Text of the last error on this context (empty if none).  Valid until the
 * next call on the context. */
const char *ptk_last_error(const ptk_ctx *ctx);

/* Set the field and the interpolation kernel.
 * u: device pointer, N*N*N*3 elements of `in_dtype` (PTK_F64 or PTK_F32),
 *    layout u[x3][x2][x1][a].  The library copies it into its own periodic,
 *    halo-padded layout in `storage_dtype` (F64, F32, BF16 or F16); the caller
 *    may free u once the call's work on `stream` has completed.
 * Storage: F64 keeps binary64; F32 rounds to nearest-even.  BF16 and F16 scale
 *    each component by its root-mean-square over the grid, s_a, stored as
 *    RNE(fl32(u_a * fl32(1/s_a))), and multiply results by fl32(s_a).
 * N: 8 <= N <= 4096.  Sums are FP64 for F64 storage and FP32 otherwise.
 * Waits for the stream when storage is BF16/F16 (it reads back s_a). */
int ptk_set_field(ptk_ctx *ctx, const void *u, int64_t N, int in_dtype, int storage_dtype,
                  const ptk_kernel *k, void *stream);

/* Per-component scale s_a of the stored field (1 for F64/F32) into host
 * float[3]. */
int ptk_get_field_scale(const ptk_ctx *ctx, float *scale3);

/* Set the field from the spectral state: the extra inverse transform that
 * particle tracking needs in a pseudo-spectral solver (Sec. 4.2, "IFT for PT"
 * in the breakdown of the overall performance).
 * spec: device pointer to the half spectrum of a real field (Sec. 2.1), N x N x
 *    (N/2+1) modes in the order [k2][k3][k1][a] -- directions 2 and 3
 *    transposed against the grid's [x3][x2][x1], as in the slab layout of
 *    Sec. 3.2 -- each complex number a (re, im) pair of `in_dtype` (PTK_F64 or
 *    PTK_F32).  Wave numbers: k1 = index (0 .. N/2); k2, k3 = index up to N/2,
 *    index - N above.  Not modified; may be freed once the call's work on
 *    `stream` has completed.
 * kind PTK_SPEC_VELOCITY: spec holds the velocity amplitudes u^(k).
 * kind PTK_SPEC_VORTICITY: spec holds the vorticity w^(k); the Biot-Savart law
 *    of Sec. 2.1 gives u^(k) = i k x w^(k) / |k|^2, with u^(0) = 0 and u^ = 0
 *    on every mode with some index equal to N/2 (no signed wave number there).
 * The grid field is the Fourier series u_a(x) = sum over all k of
 *    u^_a(k) exp(i k.x) at the nodes x = delta (j1, j2, j3) (the modes with
 *    k1 < 0 being the complex conjugates of the stored ones), computed by an
 *    inverse real FFT in the precision of in_dtype (rocFFT), then stored as by
 *    ptk_set_field (same storage types, scale and kernel rules).  The k1 = 0
 *    and k1 = N/2 planes must be Hermitian, as those of a real field are
 *    (u^(-k) = conj u^(k) within the plane); otherwise the result is
 *    undefined.
 * N: even, 8 <= N <= 2048.  The library keeps a transform buffer of
 *    3 N^2 (N/2+1) complex numbers of in_dtype, one of 3 N^3 real numbers for
 *    its result and the transform's work buffer (grown, never shrunk,
 *    released by ptk_destroy).
 * Errors: PTK_EINVAL (NULL pointer, odd or out-of-range N, bad kind or
 *    dtype), PTK_EUNSUPPORTED (kernel), PTK_ENOMEM, PTK_EHIP (transform set-up
 *    or launch); on an argument error the context is unchanged. */
enum { PTK_SPEC_VELOCITY = 0, PTK_SPEC_VORTICITY = 1, PTK_GRID = 2 };
int ptk_set_field_spectral(ptk_ctx *ctx, const void *spec, int64_t N, int in_dtype, int kind,
                           int storage_dtype, const ptk_kernel *k, void *stream);

/* The field of the end of the next time step, for a tracer step in a field
 * that changes during the step (Eq. "tracers" with u = u(x, t); in the paper's
 * loop the solver advances, the extra inverse transform of Sec. 4.2 gives the
 * new grid velocity, and the particles step from the old time to the new).
 * src: device pointer, in the form `form`:
 *   PTK_GRID: grid values u[x3][x2][x1][a] as for ptk_set_field;
 *   PTK_SPEC_VELOCITY / PTK_SPEC_VORTICITY: a half spectrum as for
 *   ptk_set_field_spectral (N even, N <= 2048).
 * N must equal the current field's; the field is stored with the current
 * field's kernel and storage type (its own per-component scale for 16-bit
 * storage) beside the current field, which it does not replace.  A new
 * current field (ptk_set_field, ptk_set_field_spectral) discards it.
 * Errors: PTK_ENOFIELD (no current field), PTK_EINVAL, PTK_ENOMEM, PTK_EHIP. */
int ptk_set_field_next(ptk_ctx *ctx, const void *src, int64_t N, int in_dtype, int form, void *stream);

/* Copy of the stored field without its halo into u (device, N*N*N*3 elements
 * of out_dtype, PTK_F64 or PTK_F32, layout u[x3][x2][x1][a]): the stored
 * values converted exactly.  16-bit storage returns its values unscaled
 * (multiply component a by ptk_get_field_scale's s_a for u_a).  Asynchronous
 * on `stream`.  Errors: PTK_ENOFIELD, PTK_EINVAL. */
int ptk_get_field(ptk_ctx *ctx, void *u, int out_dtype, void *stream);

/* Steps 1-3 of the interpolation algorithm (Sec. 2.2) for every coordinate:
 * Xtilde = X mod 2*pi; cell c = floor(Xtilde/delta); offset t = Xtilde/delta - c
 * in [0,1).  Fixed binary64 sequence per coordinate x (no fused operations):
 *   q = floor(x / L); y = x - L*q; if (y < 0) y += L; if (y >= L) y = 0;
 *   s = y * invd; c = floor(s); t = s - c; if (c == N) { c = 0; t = 0; }
 * with L = fl64(2*pi), invd = fl64(N / L).
 * X: device [Np][3] binary64.  cell: device int32 [Np][3].  t: device binary64
 * [Np][3] or NULL.  Requires a field (for N). */
int ptk_locate(ptk_ctx *ctx, const double *X, int64_t Np, int32_t *cell, double *t, void *stream);

/* Interpolate the field at Np positions (Eq. "triple_sum", indices modulo N).
 * X: device [Np][3] binary64.  out: device [Np][3] of out_dtype (PTK_F64 or
 * PTK_F32), in the order of X.  Internally particles are binned by cell with a
 * stable sort (tile columns cut into x3 windows, see ptk_binning_info), as the
 * paper groups particles by x3 slice (Sec. 3.3.1). */
int ptk_interpolate(ptk_ctx *ctx, const double *X, int64_t Np, void *out, int out_dtype,
                    void *stream);

/* Interpolate the field and its gradient: the same sum with the kernel
 * replaced by its derivative on the differentiated axis, times 1/delta.
 * u_out: device [Np][3] or NULL; grad: device [Np][3][3], grad[p][a][b] =
 * d u_a/d x_b; both of out_dtype and in the order of X. */
int ptk_interpolate_gradient(ptk_ctx *ctx, const double *X, int64_t Np, void *u_out, void *grad,
                             int out_dtype, void *stream);

/* Interpolation for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation, kernels and results as ptk_interpolate, with every
 * scratch buffer (sort keys and values, histograms, scan partials, bin
 * offsets) carved out of a fixed 32 MiB array in the library's own code object
 * instead of the context's growable scratch.  The call allocates and frees
 * nothing; the caller passes X and out as for ptk_interpolate (the field must
 * have been set before).  Limit: the scratch of Np particles on the field's
 * bins must fit the array (about 16 bytes per particle plus 4 per bin: some
 * 1.6 million particles on a 1024^3 grid); larger calls return PTK_EINVAL
 * with the size they need.  Every GPU holds one copy of the array until the
 * process ends, shared by all contexts and calls on that GPU: calls that may
 * overlap in time on one GPU (other streams, other host threads) race and
 * must be ordered by the caller.  ptk_get_binning reports no binning after
 * this call. */
int ptk_interpolate_noalloc(ptk_ctx *ctx, const double *X, int64_t Np, void *out, int out_dtype, void *stream);

/* Advance tracers dX/dt = u(X) (Eq. "tracers") by nsteps steps of dt in the
 * frozen field.
 * X: device [Np][3] binary64, in/out.  The state is the position itself,
 *    not wrapped: the reduction modulo 2*pi is step 1 of each interpolation
 *    (Sec. 2.2), so a returned trajectory keeps its crossings of the periodic
 *    faces (|x| must stay below 2^50).
 * scheme PTK_EULER: X <- X + dt u(X).
 * scheme PTK_HEUN:  k1 = u(X); Xs = X + dt k1; k2 = u(Xs);
 *                   X <- X + (0.5 dt)(k1 + k2).
 * schemes PTK_AB2, PTK_AB3, PTK_AB4 (Adams-Bashforth of order k = 2, 3, 4,
 *    the paper's multi-step integration, Sec. 2.2):
 *      X <- X + dt (b_0 u_n + b_1 u_{n-1} + ... + b_{k-1} u_{n-k+1}),
 *    b = (3/2, -1/2), (23/12, -16/12, 5/12), (55/24, -59/24, 37/24, -9/24),
 *    summed in that order; while fewer than k-1 past velocities are stored the
 *    step uses the highest order they allow (Euler first).  rhs_hist: device
 *    [k][Np][3] holding the last k velocities, most recent first (binary64
 *    for F64 storage, else FP32), in the order of X; *hist_len (host, 0..k)
 *    says how many entries are valid and is updated, so a run can resume.
 *    rhs_hist/hist_len may be NULL for Euler and Heun.
 * Every update is separately rounded binary64.
 * grad_out: device [Np][3][3] (binary64 for F64 storage, else FP32) or NULL;
 *    if given, the last step also evaluates the gradient at its start
 *    position, and on return grad_out holds it (the steps before it evaluate
 *    the velocity only; a caller that samples the gradient along the
 *    trajectory at every step advances one step per call, e.g. through
 *    ptk_particles_advance).  At a step that evaluates the gradient the
 *    velocity comes from the value + gradient kernel, whose sums are ordered
 *    differently from the value kernel's (the results can differ in the last
 *    bits): runs agree bit for bit when they request the gradient at the same
 *    steps.
 * Particles are re-binned after every position update to the stable order of
 * their new bins (only the particles whose bin changed are sorted, then merged
 * with the others) and kept in bin order internally; results are returned in
 * the order of X. */
int ptk_advance_particles(ptk_ctx *ctx, double *X, int64_t Np, void *rhs_hist, int *hist_len,
                          int scheme, double dt, int nsteps, void *grad_out, void *stream);

/* Particles kept in the library between advance calls, for a field that
 * changes between steps: in the paper's loop each step of the fluid solver is
 * followed by a tracking step on the new velocity (the extra inverse transform
 * of Sec. 4.2, here ptk_set_field_spectral), and the particle state (positions
 * and the Adams-Bashforth history, the *state* and *rhs* arrays of Sec. 3.3.1)
 * persists across steps.  ptk_particles_load sorts the caller's particles into
 * bin order once; ptk_particles_advance steps them on the current field with
 * the same schemes, arithmetic and results as ptk_advance_particles, without
 * its per-call sort, gather and final scatter; ptk_particles_store writes them
 * back in the caller's order.  Fields may be set between the calls (same N;
 * with a history loaded, a storage type of the same velocity precision).
 * The loaded state lives in the context's advance buffers: a call of
 * ptk_advance_particles or a new load replaces it.  ptk_interpolate and the
 * learned-form calls leave it alone.
 *
 * ptk_particles_load: X device [Np][3] binary64 (any real values with
 *    |x| < 2^50, kept as they are; the cells come from ptk_locate's reduction); hist_depth 0 (no history: Euler, Heun) or the
 *    Adams-Bashforth order 2..4 the history is for; rhs_hist device
 *    [hist_depth][Np][3] of the current storage's velocity type, caller order,
 *    its first hist_len (0..hist_depth) entries valid (may be NULL when
 *    hist_len = 0).  X and rhs_hist are not kept: they may be reused once the
 *    call's work on the stream has completed.  Non-finite positions give
 *    PTK_EDOMAIN (the state is then not loaded).
 * ptk_particles_advance: scheme as in ptk_advance_particles (an
 *    Adams-Bashforth scheme must match hist_depth; Euler and Heun leave a
 *    loaded history alone); grad_out as there (caller order, the last step's).
 *    PTK_EINVAL without a loaded state, with a field of another N, or with a
 *    storage type whose velocity precision differs from the loaded history's.
 * ptk_particles_store: X device [Np][3] (positions, caller order); with a
 *    history loaded, rhs_hist [hist_depth][Np][3] and *hist_len receive it.
 *    The state stays loaded. */
int ptk_particles_load(ptk_ctx *ctx, const double *X, int64_t Np, const void *rhs_hist, int hist_len,
                       int hist_depth, void *stream);
int ptk_particles_advance(ptk_ctx *ctx, int scheme, double dt, int nsteps, void *grad_out, void *stream);
int ptk_particles_store(ptk_ctx *ctx, double *X, void *rhs_hist, int *hist_len, void *stream);

/* Orientation of axisymmetric ellipsoids, a second particle type (Sec. 2.2
 * names ellipsoids among the particle types; the equation is Jeffery's,
 * 1922): the loaded particles carry unit axes p that turn with the local
 * velocity gradient A[a][b] = du_a/dx_b interpolated at the particle,
 *   dp/dt = W p + shape (S p - (p . S p) p),  S = (A + A^T)/2, W = (A - A^T)/2,
 * shape = (r^2 - 1)/(r^2 + 1) for the axis ratio r (0 spheres, 1 thin rods,
 * -1 flat discs).  Once set, ptk_particles_advance and
 * ptk_particles_step_next_field advance the axes with the positions' scheme:
 * every stage evaluates the gradient at its own position (Heun's second stage
 * then uses the value + gradient kernel), the axis rhs is FP64, an
 * Adams-Bashforth axis history is kept like the velocity history (its own
 * [k][Np][3] FP64 buffer), and p is normalized to unit length at the end of
 * each step.
 * ptk_particles_set_orientation: p device [Np][3] FP64 in the caller's order
 *    (unit vectors); p_hist device [k][Np][3] FP64 with the first hist_len
 *    entries valid, where hist_len must equal the loaded position history's
 *    length (0 without one).  Needs loaded particles; a new load drops the axes.
 * ptk_particles_get_orientation: the axes (and their history) in the caller's
 *    order.
 * Errors: PTK_EINVAL (nothing loaded, no axes set, shape outside [-1, 1],
 *    NULL pointers, history length). */
int ptk_particles_set_orientation(ptk_ctx *ctx, const double *p, const double *p_hist, int hist_len, double shape,
                                  void *stream);
int ptk_particles_get_orientation(ptk_ctx *ctx, double *p, double *p_hist, void *stream);

/* Inertial particles (NEXT-4; Sec. 2.2 names them among the particle types
 * without their equation): small heavy particles under linear (Stokes) drag,
 * dX/dt = V, dV/dt = (u(X) - V)/tau with response time tau.  Once set,
 * ptk_particles_advance and ptk_particles_step_next_field move the loaded
 * particles with their own velocities V instead of u, and V with the drag:
 * the pair (X, V) takes the scheme of the call (Euler; Heun with the
 * predictor X + dt V, V + dt r1 and the drag r2 at the predicted position and
 * velocity; AB2-AB4 with two histories of the position history's length,
 * the earlier velocities and the earlier drag terms, [k][Np][3] FP64 each).
 * Every stage interpolates u at its own position; V and the drag are FP64.
 * A particle set carries either axes or inertia: setting one drops the other.
 * ptk_particles_set_inertia: V device [Np][3] FP64 in the caller's order;
 *    v_hist and r_hist device [k][Np][3] FP64 with the first hist_len entries
 *    valid, where hist_len must equal the loaded position history's length
 *    (0 without one); tau > 0.  Needs loaded particles; a new load drops the
 *    inertia.
 * ptk_particles_get_inertia: V and its two histories in the caller's order.
 * Errors: PTK_EINVAL (nothing loaded, no inertia set, tau not positive and
 *    finite, NULL pointers, history length). */
int ptk_particles_set_inertia(ptk_ctx *ctx, const double *V, const double *v_hist, const double *r_hist,
                              int hist_len, double tau, void *stream);
int ptk_particles_get_inertia(ptk_ctx *ctx, double *V, double *v_hist, double *r_hist, void *stream);

/* In-order particle state files: checkpoint / restart and output for
 * post-processing (Sec. 3.4: the particles are written in the original order
 * given as input, so that outputs are consistent from one to the next whatever
 * order the library keeps them in).
 * ptk_particles_save writes the loaded state to `path` (host file, replaced):
 * a 64-byte header -- "PTKSTATE", uint32 version 1, uint32 flags (bit 0: axes
 * follow, bit 1: inertia follows), int64 Np, int32 history depth k, int32
 * valid history entries h, int32 bytes per history component (8 or 4), int32
 * grid N, float64 axis shape, float64 response time tau (inertia; else 0), 8
 * reserved bytes, little-endian -- then, in the caller's order, positions
 * [Np][3] float64, the history [h][Np][3], and with axes the axes [Np][3]
 * float64 and their history [h][Np][3] float64, or with inertia the
 * velocities [Np][3] float64, their history and the drag history
 * ([h][Np][3] float64 each).  Waits for the
 * stream; goes through the device (a staging copy of the state) and one
 * 32 MiB pinned host buffer.
 * ptk_particles_restore makes a file's state the loaded state, as
 * ptk_particles_load (and ptk_particles_set_orientation or _set_inertia) would from those
 * arrays; needs a field with the file's N (and, with a history, a storage
 * type of its velocity precision).  A run restored from a file continues bit
 * for bit as the run that saved it.
 * Errors: PTK_EIO (file cannot be opened, written or read; bad header),
 * PTK_EINVAL, PTK_ENOFIELD, PTK_ENOMEM, PTK_EHIP, PTK_EDOMAIN. */
int ptk_particles_save(ptk_ctx *ctx, const char *path, void *stream);
int ptk_particles_restore(ptk_ctx *ctx, const char *path, void *stream);

/* One Heun step of the loaded particles from t to t + dt whose stages see the
 * fields of their own times: the current field (time t) and the next field
 * (time t + dt, ptk_set_field_next):
 *   k1 = u(X, t); Xs = X + dt k1; k2 = u(Xs, t + dt); X <- X + (0.5 dt)(k1 + k2).
 * Same arithmetic, re-binning and state handling as ptk_particles_advance with
 * PTK_HEUN (a loaded Adams-Bashforth history is left alone); grad_out as there
 * (at X, on the current field).  Afterwards the next field is the current one
 * (its buffer swapped in; no copy) and no next field is set.  The Heun stages
 * fall exactly on the two times, so no interpolation in time is needed.
 * Errors: PTK_EINVAL (nothing loaded, other N), PTK_ENOFIELD (no current or
 * next field). */
int ptk_particles_step_next_field(ptk_ctx *ctx, double dt, void *grad_out, void *stream);

/* Binning of the last ptk_interpolate / ptk_interpolate_gradient call:
 * number of particles, number of bins, tile edge T and window depth W (cells).
 * Bins are tile columns of T x T cells in (x1, x2), each cut along x3 into
 * windows of W cell layers; bin of cell c:
 *   key = ((c2/T) * ntx + c1/T) * nw + c3/W,  ntx = ceil(N/T), nw = ceil(N/W),
 * so within a column particles are ordered along x3 like the paper's slices.
 * T is 12 and W is 5 for every storage type (with I = 8 the W + I - 1 = 12
 * planes a window touches fill the LDS ring). */
int ptk_binning_info(const ptk_ctx *ctx, int64_t *np, int64_t *n_bins, int *tile, int *window);

/* Copy that binning to device buffers: perm[k] (uint32 [np]) = index in X of
 * the k-th particle in bin order (a stable sort of the keys), offsets (uint32
 * [n_bins+1]) with offsets[b] = number of particles with key < b and
 * offsets[n_bins] = np (the paper's offset array, Sec. 3.3.1). */
int ptk_get_binning(ptk_ctx *ctx, uint32_t *perm, uint32_t *offsets, void *stream);

/* Kernel timing, a tracing aid.  While enabled, the library brackets its main
 * launch sequences with HIP events on the call's stream and accumulates their
 * durations per kind:
 *   PTK_T_INTERP       interpolation kernel, values only
 *   PTK_T_INTERP_GRAD  interpolation kernel with gradient
 *   PTK_T_SORT         stable radix sort + bin offsets
 *   PTK_T_KEYS         bin keys of caller positions
 *   PTK_T_UPDATE       position update (+ keys of the new positions)
 *   PTK_T_PERMUTE      gathers/scatters of particle state between orders
 *   PTK_T_LEARNED      learned-form inference kernel (features, L4 sum, network)
 *   PTK_T_IFT          spectral set-up: spectrum reorder (and Biot-Savart) and
 *                      the inverse FFT (the field pack is not included)
 * ptk_timing_enable(ctx, 1) starts (and clears) the accumulators, 0 stops.
 * ptk_timing_read waits for the recorded events, adds their durations to the
 * accumulators and copies them out: ms[PTK_T_COUNT] (milliseconds) and
 * launches[PTK_T_COUNT] (number of timed sequences); either may be NULL. */
enum { PTK_T_INTERP = 0, PTK_T_INTERP_GRAD = 1, PTK_T_SORT = 2, PTK_T_KEYS = 3, PTK_T_UPDATE = 4,
       PTK_T_PERMUTE = 5, PTK_T_LEARNED = 6, PTK_T_IFT = 7, PTK_T_COUNT = 8 };
int ptk_timing_enable(ptk_ctx *ctx, int enable);
int ptk_timing_read(ptk_ctx *ctx, double *ms, int64_t *launches);

/* ---- Learned correction form ------------------------------------------
 * Beside the paper's weighted sum: a network of 195 -> 128 -> 128 -> 3
 * units predicts, from the 4 x 4 x 4 stencil of the I = 4 Lagrange kernel and
 * the in-cell offsets, the difference between the context's kernel (the
 * "wide" kernel, e.g. the I = 8 C2 spline) and the I = 4 Lagrange interpolant:
 * u ~ u_L4 + y.  Needs FP32 field storage and a wide kernel with I >= 4.
 *
 * Features of a particle in cell c with offsets t (steps 1-3 of Sec. 2.2):
 * BF16 numbers (round to nearest even), f = ((k3*4 + k2)*4 + k1)*3 + a for
 * the stored field component a at node c + (k - 1) (k in 0..3 per axis,
 * indices modulo N), then t1, t2, t3 (rounded to FP32, then to BF16) at f =
 * 192..194.  Rows are PTK_LEARNED_FEAT_PITCH = 200 BF16 wide (400 bytes);
 * entries 195..199 are zero.
 * Network: z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2, h2 = silu(z2),
 * y = W3 h2 + b3, silu(z) = z / (1 + exp(-z)).  Parameters are one FP32
 * vector of PTK_LEARNED_NPARAMS numbers: W1[128][195], b1[128], W2[128][128],
 * b2[128], W3[3][128], b3[3].  The two hidden-layer products (and the
 * backward products through them) take BF16 operands -- x, W1, h1, W2; dz2,
 * h1, W2, dz1, x -- with FP32 sums on the matrix cores; the rest is FP32. */
#define PTK_LEARNED_NFEAT 195
#define PTK_LEARNED_FEAT_PITCH 200
#define PTK_LEARNED_NPARAMS 41987

/* Training pairs at Np positions: feat (device, uint16 BF16 bits
 * [Np][PTK_LEARNED_FEAT_PITCH]) and target (device FP32 [Np][3]) =
 * u_wide(X) - u_L4(X), both sums in FP32.  Either output may be NULL. */
int ptk_learned_make_pairs(ptk_ctx *ctx, const double *X, int64_t Np, uint16_t *feat, float *target,
                           void *stream);

/* Load the FP32 master parameters (host, PTK_LEARNED_NPARAMS floats) and
 * reset the optimiser state (moments and step count).  Synchronous. */
int ptk_learned_set_params(ptk_ctx *ctx, const float *params);

/* Copy the FP32 master parameters to host memory.  Synchronous. */
int ptk_learned_get_params(ptk_ctx *ctx, float *params);

/* Mean-square loss over n pairs and its gradient with respect to the
 * parameters, without an update: loss (device FP32 [1]) = mean over rows and
 * the 3 components of (y - target)^2; grad (device FP32 [PTK_LEARNED_NPARAMS],
 * parameter layout).  n: multiple of 64, 64 <= n <= 16384. */
int ptk_learned_loss_grad(ptk_ctx *ctx, const uint16_t *feat, const float *target, int64_t n,
                          float *loss, float *grad, void *stream);

/* Optimiser settings: Adam (Kingma and Ba) with bias correction, step size
 * lr * (1 + cos(pi s / S)) / 2 at step s of S = epochs * (n / batch). */
typedef struct {
  int epochs;
  int batch;    /* multiple of 64, 64 .. 16384 */
  float lr;
  float beta1;
  float beta2;
  float eps;
} ptk_train_config;

/* Train on n pairs: epochs passes over consecutive batches (a trailing
 * partial batch is dropped), one Adam step per batch; the optimiser state
 * continues from the last set_params/train call.  loss_curve: device FP32
 * [epochs * (n / batch)] receiving each step's batch loss, or NULL. */
int ptk_learned_train(ptk_ctx *ctx, const uint16_t *feat, const float *target, int64_t n,
                      const ptk_train_config *cfg, float *loss_curve, void *stream);

/* Learned interpolation: out (device FP32 [Np][3], in the order of X) =
 * u_L4(X) + y(features).  Audit: the wide kernel is evaluated at particles
 * 0, k, 2k, ... (k = round(1/audit_frac), audit_frac in (0, 1]); *audit_rms
 * (host) receives sqrt(sum |out - u_wide|^2 / sum |u_wide|^2) over them, and
 * if it exceeds tol_rel_rms the whole output is recomputed with the wide
 * kernel and *fell_back (host) is set to 1 (else 0).  Waits for the stream
 * (it reads the audit back). */
int ptk_interpolate_learned(ptk_ctx *ctx, const double *X, int64_t Np, float *out, double audit_frac,
                            double tol_rel_rms, double *audit_rms, int *fell_back, void *stream);

/* Host-only self-test of the library's internal checks (the scratch capacity
 * guard that every launch sequence passes before it writes scratch, the byte
 * cap of PTK_TEST_MAX_BYTES, the decoding of the device status word).  Needs
 * no device and no context; returns PTK_OK when every check behaves as
 * documented, PTK_EINTERNAL otherwise. */
int ptk_selftest(void);

#ifdef __cplusplus
}
#endif

#endif /* PTK_H */
