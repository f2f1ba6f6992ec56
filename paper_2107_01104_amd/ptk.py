"""Python binding of libptk (include/ptk.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch device
tensors to pointers, passes torch's current HIP stream, and turns return codes
into exceptions.  Importing it without a built ``libptk.so`` raises: there is no
fallback path.

Low-level functions carry the C names (``ptk_create``, ``ptk_set_field``, ...);
``Context`` wraps them for convenience.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptk.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
LAGRANGE, SPLINE = 0, 1
EULER, HEUN, AB2, AB3, AB4 = 1, 2, 3, 4, 5
AB_ORDER = {AB2: 2, AB3: 3, AB4: 4}
OK, EINVAL, ENOFIELD, ENOMEM, EHIP, EDOMAIN, EUNSUPPORTED, EINTERNAL, EIO = 0, -1, -2, -3, -4, -5, -6, -7, -8
TIMERS = ["interp", "interp_grad", "sort", "keys", "update", "permute", "learned", "ift"]
SPEC_VELOCITY, SPEC_VORTICITY, GRID = 0, 1, 2
LEARNED_NFEAT, LEARNED_FEAT_PITCH, LEARNED_NPARAMS = 195, 200, 41987

EXPORTS = ["ptk_kernel_table", "ptk_kernel_table_centred", "ptk_create", "ptk_destroy", "ptk_last_error", "ptk_set_field", "ptk_get_field_scale",
           "ptk_set_field_spectral", "ptk_set_field_next", "ptk_get_field", "ptk_particles_load",
           "ptk_particles_advance", "ptk_particles_store", "ptk_particles_step_next_field",
           "ptk_particles_set_orientation", "ptk_particles_get_orientation", "ptk_particles_set_inertia",
           "ptk_particles_get_inertia", "ptk_particles_save",
           "ptk_particles_restore",
           "ptk_locate", "ptk_interpolate", "ptk_interpolate_gradient", "ptk_advance_particles",
           "ptk_binning_info", "ptk_get_binning", "ptk_timing_enable", "ptk_timing_read",
           "ptk_learned_make_pairs", "ptk_learned_set_params", "ptk_learned_get_params", "ptk_learned_loss_grad",
           "ptk_learned_train", "ptk_interpolate_learned", "ptk_selftest", "ptk_interpolate_noalloc"]

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2107_01104_amd/build.py` first")

lib = ctypes.CDLL(LIB_PATH)


class ptk_kernel(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int), ("I", ctypes.c_int), ("m", ctypes.c_int)]


class ptk_train_config(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_vp, _i64, _int, _dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
lib.ptk_kernel_table.argtypes = [ctypes.POINTER(ptk_kernel), _vp, _vp]
lib.ptk_kernel_table_centred.argtypes = [ctypes.POINTER(ptk_kernel), _vp, _vp, _vp, _vp]
lib.ptk_create.argtypes = [ctypes.POINTER(_vp), _int]
lib.ptk_destroy.argtypes = [_vp]
lib.ptk_destroy.restype = None
lib.ptk_last_error.argtypes = [_vp]
lib.ptk_last_error.restype = ctypes.c_char_p
lib.ptk_set_field.argtypes = [_vp, _vp, _i64, _int, _int, ctypes.POINTER(ptk_kernel), _vp]
lib.ptk_get_field_scale.argtypes = [_vp, ctypes.POINTER(ctypes.c_float)]
lib.ptk_set_field_spectral.argtypes = [_vp, _vp, _i64, _int, _int, _int, ctypes.POINTER(ptk_kernel), _vp]
lib.ptk_get_field.argtypes = [_vp, _vp, _int, _vp]
lib.ptk_set_field_next.argtypes = [_vp, _vp, _i64, _int, _int, _vp]
lib.ptk_particles_step_next_field.argtypes = [_vp, _dbl, _vp, _vp]
lib.ptk_particles_set_orientation.argtypes = [_vp, _vp, _vp, _int, _dbl, _vp]
lib.ptk_particles_get_orientation.argtypes = [_vp, _vp, _vp, _vp]
lib.ptk_particles_set_inertia.argtypes = [_vp, _vp, _vp, _vp, _int, _dbl, _vp]
lib.ptk_particles_get_inertia.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.ptk_particles_save.argtypes = [_vp, ctypes.c_char_p, _vp]
lib.ptk_particles_restore.argtypes = [_vp, ctypes.c_char_p, _vp]
lib.ptk_locate.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp]
lib.ptk_interpolate.argtypes = [_vp, _vp, _i64, _vp, _int, _vp]
lib.ptk_interpolate_gradient.argtypes = [_vp, _vp, _i64, _vp, _vp, _int, _vp]
lib.ptk_interpolate_noalloc.argtypes = [_vp, _vp, _i64, _vp, _int, _vp]
lib.ptk_advance_particles.argtypes = [_vp, _vp, _i64, _vp, ctypes.POINTER(_int), _int, _dbl, _int, _vp, _vp]
lib.ptk_particles_load.argtypes = [_vp, _vp, _i64, _vp, _int, _int, _vp]
lib.ptk_particles_advance.argtypes = [_vp, _int, _dbl, _int, _vp, _vp]
lib.ptk_particles_store.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_int), _vp]
lib.ptk_binning_info.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_int),
                                 ctypes.POINTER(_int)]
lib.ptk_get_binning.argtypes = [_vp, _vp, _vp, _vp]
lib.ptk_timing_enable.argtypes = [_vp, _int]
lib.ptk_timing_read.argtypes = [_vp, _vp, _vp]
lib.ptk_learned_make_pairs.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp]
lib.ptk_learned_set_params.argtypes = [_vp, _vp]
lib.ptk_learned_get_params.argtypes = [_vp, _vp]
lib.ptk_learned_loss_grad.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp, _vp]
lib.ptk_learned_train.argtypes = [_vp, _vp, _vp, _i64, ctypes.POINTER(ptk_train_config), _vp, _vp]
lib.ptk_interpolate_learned.argtypes = [_vp, _vp, _i64, _vp, _dbl, _dbl, ctypes.POINTER(_dbl),
                                        ctypes.POINTER(_int), _vp]
lib.ptk_selftest.argtypes = []
for _name in EXPORTS:
    if _name not in ("ptk_destroy", "ptk_last_error"):
        getattr(lib, _name).restype = _int

# the C entry points under their own names
ptk_kernel_table = lib.ptk_kernel_table
ptk_kernel_table_centred = lib.ptk_kernel_table_centred
ptk_create = lib.ptk_create
ptk_destroy = lib.ptk_destroy
ptk_last_error = lib.ptk_last_error
ptk_set_field = lib.ptk_set_field
ptk_get_field_scale = lib.ptk_get_field_scale
ptk_locate = lib.ptk_locate
ptk_interpolate = lib.ptk_interpolate
ptk_interpolate_gradient = lib.ptk_interpolate_gradient
ptk_interpolate_noalloc = lib.ptk_interpolate_noalloc
ptk_advance_particles = lib.ptk_advance_particles
ptk_binning_info = lib.ptk_binning_info
ptk_get_binning = lib.ptk_get_binning
ptk_timing_enable = lib.ptk_timing_enable
ptk_timing_read = lib.ptk_timing_read
ptk_learned_make_pairs = lib.ptk_learned_make_pairs
ptk_learned_set_params = lib.ptk_learned_set_params
ptk_learned_get_params = lib.ptk_learned_get_params
ptk_learned_loss_grad = lib.ptk_learned_loss_grad
ptk_learned_train = lib.ptk_learned_train
ptk_interpolate_learned = lib.ptk_interpolate_learned
ptk_selftest = lib.ptk_selftest


def kernel_table(family: int, I: int, m: int = 0):
    """(val, der) coefficient tables [I][I] of the library's kernel (host only)."""
    import numpy as np
    val = np.zeros((I, I))
    der = np.zeros((I, I))
    k = ptk_kernel(int(family), int(I), int(m))
    rc = lib.ptk_kernel_table(ctypes.byref(k), val.ctypes.data_as(_vp), der.ctypes.data_as(_vp))
    if rc != OK:
        raise PtkError(rc, "ptk_kernel_table failed")
    return val, der


def kernel_table_centred(family: int, I: int, m: int = 0):
    """(val, der, val32, der32) coefficient tables [I][I] in powers of
    (t - 1/2), binary64 and binary32 (host only)."""
    import numpy as np
    val, der = np.zeros((I, I)), np.zeros((I, I))
    v32, d32 = np.zeros((I, I), dtype=np.float32), np.zeros((I, I), dtype=np.float32)
    k = ptk_kernel(int(family), int(I), int(m))
    rc = lib.ptk_kernel_table_centred(ctypes.byref(k), val.ctypes.data_as(_vp), der.ctypes.data_as(_vp),
                                      v32.ctypes.data_as(_vp), d32.ctypes.data_as(_vp))
    if rc != OK:
        raise PtkError(rc, "ptk_kernel_table_centred failed")
    return val, der, v32, d32


class PtkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ptk error {code}: {msg}")
        self.code = code


_TORCH_OF = {F64: torch.float64, F32: torch.float32}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(t, dtype, shape_tail, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} must end in shape {shape_tail}")
    return t


class Context:
    """One libptk context on one device."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = lib.ptk_create(ctypes.byref(h), int(device))
        if rc != OK:
            raise PtkError(rc, "ptk_create failed")
        self._h = h
        self.storage = None
        self.N = None

    def close(self):
        if getattr(self, "_h", None):
            lib.ptk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise PtkError(rc, lib.ptk_last_error(self._h).decode())

    def set_field(self, u: torch.Tensor, family: int, I: int, m: int = 0, storage: int = F32):
        if u.dtype not in (torch.float64, torch.float32):
            raise TypeError("field must be float64 or float32")
        _dev_tensor(u, u.dtype, (3,), "u")
        N = u.shape[0]
        if tuple(u.shape) != (N, N, N, 3):
            raise ValueError("field must have shape (N, N, N, 3)")
        k = ptk_kernel(int(family), int(I), int(m))
        in_dt = F64 if u.dtype == torch.float64 else F32
        self._check(lib.ptk_set_field(self._h, _ptr(u), N, in_dt, int(storage), ctypes.byref(k),
                                      _stream(self.device)))
        self.storage, self.N = int(storage), N

    def set_field_spectral(self, spec: torch.Tensor, family: int, I: int, m: int = 0, storage: int = F32,
                           kind: int = SPEC_VELOCITY):
        """Field from its half spectrum spec[k2][k3][k1][a] (complex128 or
        complex64, shape (N, N, N//2+1, 3)): velocity amplitudes, or vorticity
        with kind=SPEC_VORTICITY (include/ptk.h, ptk_set_field_spectral)."""
        if spec.dtype not in (torch.complex128, torch.complex64):
            raise TypeError("spectrum must be complex128 or complex64")
        _dev_tensor(spec, spec.dtype, (3,), "spec")
        N = spec.shape[0]
        if spec.dim() != 4 or tuple(spec.shape) != (N, N, N // 2 + 1, 3):
            raise ValueError("spectrum must have shape (N, N, N//2+1, 3)")
        k = ptk_kernel(int(family), int(I), int(m))
        in_dt = F64 if spec.dtype == torch.complex128 else F32
        self._check(lib.ptk_set_field_spectral(self._h, _ptr(spec), N, in_dt, int(kind), int(storage),
                                               ctypes.byref(k), _stream(self.device)))
        self.storage, self.N = int(storage), N

    def set_field_next(self, src: torch.Tensor):
        """The field of the end of the next step (include/ptk.h,
        ptk_set_field_next): grid values [N][N][N][3] (float64/float32) or a
        half spectrum [N][N][N//2+1][3] (complex128/complex64) of velocity;
        pass kind=SPEC_VORTICITY through set_field_next_spectral for a
        vorticity spectrum."""
        return self._set_next(src, None)

    def set_field_next_spectral(self, spec: torch.Tensor, kind: int = SPEC_VELOCITY):
        return self._set_next(spec, int(kind))

    def _set_next(self, src, kind):
        if kind is None:
            if src.dtype not in (torch.float64, torch.float32):
                raise TypeError("grid field must be float64 or float32")
            form, in_dt = GRID, (F64 if src.dtype == torch.float64 else F32)
        else:
            if src.dtype not in (torch.complex128, torch.complex64):
                raise TypeError("spectrum must be complex128 or complex64")
            form, in_dt = kind, (F64 if src.dtype == torch.complex128 else F32)
        _dev_tensor(src, src.dtype, (3,), "src")
        self._check(lib.ptk_set_field_next(self._h, _ptr(src), src.shape[0], in_dt, form, _stream(self.device)))

    def particles_step_next_field(self, dt: float, grad_out=None):
        """One Heun step of the resident particles: first stage on the current
        field, second on the next; the next field then becomes current."""
        if grad_out is not None:
            _dev_tensor(grad_out, self.vel_dtype(), (3, 3), "grad_out")
        self._check(lib.ptk_particles_step_next_field(self._h, float(dt), _ptr(grad_out), _stream(self.device)))

    def get_field(self, dtype=torch.float64):
        """The stored field without halo, [N][N][N][3] (16-bit storage: unscaled)."""
        if dtype not in _TORCH_OF.values():
            raise TypeError("dtype must be float64 or float32")
        code = F64 if dtype == torch.float64 else F32
        if self.N is None:  # no field: the library reports it
            self._check(lib.ptk_get_field(self._h, None, code, None))
        out = torch.empty((self.N, self.N, self.N, 3), dtype=dtype, device=self.device)
        self._check(lib.ptk_get_field(self._h, _ptr(out), code, _stream(self.device)))
        return out

    def field_scale(self):
        s = (ctypes.c_float * 3)()
        self._check(lib.ptk_get_field_scale(self._h, s))
        return [s[0], s[1], s[2]]

    def vel_dtype(self):
        return torch.float64 if self.storage == F64 else torch.float32

    def locate(self, X: torch.Tensor, with_offset: bool = True):
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        cell = torch.empty((n, 3), dtype=torch.int32, device=X.device)
        t = torch.empty((n, 3), dtype=torch.float64, device=X.device) if with_offset else None
        self._check(lib.ptk_locate(self._h, _ptr(X), n, _ptr(cell), _ptr(t), _stream(self.device)))
        return (cell, t) if with_offset else cell

    def interpolate(self, X: torch.Tensor, out_dtype=torch.float32, out=None):
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        if out is None:
            out = torch.empty((n, 3), dtype=out_dtype, device=X.device)
        code = F64 if out.dtype == torch.float64 else F32
        self._check(lib.ptk_interpolate(self._h, _ptr(X), n, _ptr(out), code, _stream(self.device)))
        return out

    def interpolate_noalloc(self, X: torch.Tensor, out: torch.Tensor):
        """ptk_interpolate_noalloc: the library allocates nothing; out is the
        caller's [Np][3] float32 or float64 tensor."""
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        if out.dtype not in (torch.float32, torch.float64):
            raise TypeError("out must be float32 or float64")
        _dev_tensor(out, out.dtype, (3,), "out")
        if out.numel() // 3 != n:
            raise ValueError("out must have Np rows")
        code = F64 if out.dtype == torch.float64 else F32
        self._check(lib.ptk_interpolate_noalloc(self._h, _ptr(X), n, _ptr(out), code, _stream(self.device)))
        return out

    def interpolate_gradient(self, X: torch.Tensor, out_dtype=torch.float32, with_value: bool = True):
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        u = torch.empty((n, 3), dtype=out_dtype, device=X.device) if with_value else None
        g = torch.empty((n, 3, 3), dtype=out_dtype, device=X.device)
        code = F64 if out_dtype == torch.float64 else F32
        self._check(lib.ptk_interpolate_gradient(self._h, _ptr(X), n, _ptr(u), _ptr(g), code,
                                                 _stream(self.device)))
        return u, g

    def advance(self, X: torch.Tensor, scheme: int, dt: float, nsteps: int, hist=None, hist_len: int = 0,
                grad_out=None):
        """Advance X in place; returns the new history length (Adams-Bashforth) or 0."""
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        hl = ctypes.c_int(int(hist_len))
        if hist is not None:
            _dev_tensor(hist, self.vel_dtype(), (3,), "rhs_hist")
            k = AB_ORDER.get(int(scheme), 2)
            if tuple(hist.shape) != (k, n, 3):
                raise ValueError(f"rhs_hist must have shape ({k}, Np, 3)")
        if grad_out is not None:
            _dev_tensor(grad_out, self.vel_dtype(), (3, 3), "grad_out")
        self._check(lib.ptk_advance_particles(self._h, _ptr(X), n, _ptr(hist),
                                              ctypes.byref(hl) if hist is not None else None,
                                              int(scheme), float(dt), int(nsteps), _ptr(grad_out),
                                              _stream(self.device)))
        return hl.value

    # ---- particles kept in the library between advance calls
    def particles_load(self, X: torch.Tensor, hist=None, hist_len: int = 0, hist_depth: int = 0):
        """Load X ([Np][3] float64) and optionally an Adams-Bashforth history
        ([hist_depth][Np][3], hist_len valid entries) as the resident state."""
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        if hist is not None:
            _dev_tensor(hist, self.vel_dtype(), (3,), "rhs_hist")
            if tuple(hist.shape) != (int(hist_depth), n, 3):
                raise ValueError(f"rhs_hist must have shape ({hist_depth}, Np, 3)")
        self._check(lib.ptk_particles_load(self._h, _ptr(X), n, _ptr(hist), int(hist_len), int(hist_depth),
                                           _stream(self.device)))

    def particles_advance(self, scheme: int, dt: float, nsteps: int, grad_out=None):
        """Step the resident particles on the current field."""
        if grad_out is not None:
            _dev_tensor(grad_out, self.vel_dtype(), (3, 3), "grad_out")
        self._check(lib.ptk_particles_advance(self._h, int(scheme), float(dt), int(nsteps), _ptr(grad_out),
                                              _stream(self.device)))

    def particles_store(self, X: torch.Tensor, hist=None):
        """Write the resident positions (and history) in caller order; returns
        the history length."""
        _dev_tensor(X, torch.float64, (3,), "X")
        if hist is not None:
            _dev_tensor(hist, self.vel_dtype(), (3,), "rhs_hist")
        hl = ctypes.c_int(0)
        self._check(lib.ptk_particles_store(self._h, _ptr(X), _ptr(hist), ctypes.byref(hl),
                                            _stream(self.device)))
        return hl.value

    def particles_set_orientation(self, p: torch.Tensor, shape: float, hist=None, hist_len: int = 0):
        """Unit axes p ([Np][3] float64, caller order) of the loaded particles,
        turned by Jeffery's equation with the given shape factor in later
        steps; an Adams-Bashforth axis history ([k][Np][3] float64) with as
        many valid entries as the position history."""
        _dev_tensor(p, torch.float64, (3,), "p")
        if hist is not None:
            _dev_tensor(hist, torch.float64, (3,), "p_hist")
        self._check(lib.ptk_particles_set_orientation(self._h, _ptr(p), _ptr(hist), int(hist_len), float(shape),
                                                      _stream(self.device)))

    def particles_get_orientation(self, p: torch.Tensor, hist=None):
        _dev_tensor(p, torch.float64, (3,), "p")
        if hist is not None:
            _dev_tensor(hist, torch.float64, (3,), "p_hist")
        self._check(lib.ptk_particles_get_orientation(self._h, _ptr(p), _ptr(hist), _stream(self.device)))

    def particles_set_inertia(self, V: torch.Tensor, tau: float, v_hist=None, r_hist=None, hist_len: int = 0):
        """Velocities V ([Np][3] float64, caller order) of the loaded particles,
        which from then on move with V under linear drag, dV/dt = (u - V)/tau;
        with an Adams-Bashforth history, the earlier velocities and drag terms
        ([k][Np][3] float64 each) with as many valid entries as the position
        history.  Replaces axes set before."""
        _dev_tensor(V, torch.float64, (3,), "V")
        for name, h in (("v_hist", v_hist), ("r_hist", r_hist)):
            if h is not None:
                _dev_tensor(h, torch.float64, (3,), name)
        self._check(lib.ptk_particles_set_inertia(self._h, _ptr(V), _ptr(v_hist), _ptr(r_hist), int(hist_len),
                                                  float(tau), _stream(self.device)))

    def particles_get_inertia(self, V: torch.Tensor, v_hist=None, r_hist=None):
        _dev_tensor(V, torch.float64, (3,), "V")
        for name, h in (("v_hist", v_hist), ("r_hist", r_hist)):
            if h is not None:
                _dev_tensor(h, torch.float64, (3,), name)
        self._check(lib.ptk_particles_get_inertia(self._h, _ptr(V), _ptr(v_hist), _ptr(r_hist),
                                                  _stream(self.device)))

    def particles_save(self, path: str):
        """Write the loaded state to a file in the caller's order."""
        self._check(lib.ptk_particles_save(self._h, os.fsencode(path), _stream(self.device)))

    def particles_restore(self, path: str):
        """Make a state file's particles the loaded state."""
        self._check(lib.ptk_particles_restore(self._h, os.fsencode(path), _stream(self.device)))

    def binning(self):
        """(perm, offsets, tile, window) of the last interpolate call."""
        np_, nb, tile, win = _i64(), _i64(), _int(), _int()
        self._check(lib.ptk_binning_info(self._h, ctypes.byref(np_), ctypes.byref(nb), ctypes.byref(tile),
                                         ctypes.byref(win)))
        perm = torch.empty(max(np_.value, 1), dtype=torch.int32, device=self.device)
        off = torch.empty(nb.value + 1, dtype=torch.int32, device=self.device)
        self._check(lib.ptk_get_binning(self._h, _ptr(perm), _ptr(off), _stream(self.device)))
        return perm[: np_.value], off, tile.value, win.value

    def timing(self, enable: bool):
        self._check(lib.ptk_timing_enable(self._h, int(bool(enable))))

    def timing_read(self):
        """{kind: (total_ms, launches)} accumulated since timing was enabled."""
        import numpy as np
        ms = np.zeros(len(TIMERS))
        cnt = np.zeros(len(TIMERS), dtype=np.int64)
        self._check(lib.ptk_timing_read(self._h, ms.ctypes.data_as(_vp), cnt.ctypes.data_as(_vp)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(TIMERS)}

    # ---- learned correction form
    def learned_make_pairs(self, X: torch.Tensor, features: bool = True, targets: bool = True):
        """(feat uint16 [Np, 200] BF16 bits, target float32 [Np, 3]) at positions X."""
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        feat = torch.empty((n, LEARNED_FEAT_PITCH), dtype=torch.int16, device=X.device) if features else None
        tgt = torch.empty((n, 3), dtype=torch.float32, device=X.device) if targets else None
        self._check(lib.ptk_learned_make_pairs(self._h, _ptr(X), n, _ptr(feat), _ptr(tgt), _stream(self.device)))
        return feat, tgt

    def learned_set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if p.size != LEARNED_NPARAMS:
            raise ValueError(f"expected {LEARNED_NPARAMS} parameters")
        self._check(lib.ptk_learned_set_params(self._h, p.ctypes.data_as(_vp)))

    def learned_get_params(self):
        import numpy as np
        p = np.empty(LEARNED_NPARAMS, dtype=np.float32)
        self._check(lib.ptk_learned_get_params(self._h, p.ctypes.data_as(_vp)))
        return p

    def learned_loss_grad(self, feat: torch.Tensor, target: torch.Tensor):
        """(loss float32 [1], grad float32 [41987]) of one batch, no update."""
        _dev_tensor(feat, torch.int16, (LEARNED_FEAT_PITCH,), "feat")
        _dev_tensor(target, torch.float32, (3,), "target")
        n = feat.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        grad = torch.empty(LEARNED_NPARAMS, dtype=torch.float32, device=feat.device)
        self._check(lib.ptk_learned_loss_grad(self._h, _ptr(feat), _ptr(target), n, _ptr(loss), _ptr(grad),
                                              _stream(self.device)))
        return loss, grad

    def learned_train(self, feat: torch.Tensor, target: torch.Tensor, epochs: int, batch: int = 4096,
                      lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        """Adam over consecutive batches; returns the per-step loss curve (float32 tensor)."""
        _dev_tensor(feat, torch.int16, (LEARNED_FEAT_PITCH,), "feat")
        _dev_tensor(target, torch.float32, (3,), "target")
        n = feat.shape[0]
        steps = int(epochs) * (n // int(batch))
        curve = torch.empty(max(steps, 1), dtype=torch.float32, device=feat.device)
        cfg = ptk_train_config(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps))
        self._check(lib.ptk_learned_train(self._h, _ptr(feat), _ptr(target), n, ctypes.byref(cfg), _ptr(curve),
                                          _stream(self.device)))
        return curve[:steps]

    def interpolate_learned(self, X: torch.Tensor, audit_frac: float = 1e-3, tol_rel_rms: float = 1e-4,
                            out=None):
        """(out float32 [Np, 3], audit_rms, fell_back)."""
        _dev_tensor(X, torch.float64, (3,), "X")
        n = X.numel() // 3
        if out is None:
            out = torch.empty((n, 3), dtype=torch.float32, device=X.device)
        a = _dbl()
        fb = _int()
        self._check(lib.ptk_interpolate_learned(self._h, _ptr(X), n, _ptr(out), float(audit_frac),
                                                float(tol_rel_rms), ctypes.byref(a), ctypes.byref(fb),
                                                _stream(self.device)))
        return out, a.value, bool(fb.value)
